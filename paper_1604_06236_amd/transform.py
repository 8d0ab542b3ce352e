"""Python binding of the block transform: the C-ABI entry points on torch tensors.

Argument marshalling only: every arithmetic step runs in the HIP library.
torch supplies device memory (outputs, workspace) and the current stream.

Shapes: coefficient / sample tensors are complex64 [B, N] (N = K*M), taps are
float32 [N] (shared) or [B, N] (one filter per block), all contiguous on the
same GPU.  The operators (per block, omega = exp(j 2 pi / N)):

  transform_forward          y_u  = sum_n taps_n S_n omega^{+nu}          (eq. (6) on u/N; eq. (7) at u = Mq)
  transform_inverse          S_n  = (N taps_n)^{-1} sum_u y_u omega^{-nu}  (eq. (31), any nonzero filter)
  transform_adjoint          Sbar = taps . W,  tapbar = Re(conj(S) W),  W_n = sum_u ybar_u omega^{-nu}
  transform_inverse_adjoint  ybar_u = sum_n omega^{+nu} g_n/(N taps_n),  tapbar = -Re(conj(g) Shat)/taps
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from . import _native as nat


_RAGGED_CHUNK = 0      # tiles per ragged work item (0: automatic)


def load_schedules(path: Optional[str] = None) -> bool:
    """Apply autotuned schedule choices from a JSON file ($BT_SCHEDULES, or
    schedules.json next to this module): per-(K, M) schedules go to the library,
    the ragged work-item size ("ragged_chunk_tiles") to RaggedPlan and the ragged
    per-class prefetch choices ("ragged_prefetch": {"KxM": [forward, output side,
    tap gradient]}, 0 off / 1 on) to the library.  Returns True when a file was
    applied."""
    import json
    import os
    global _RAGGED_CHUNK
    path = path or os.environ.get("BT_SCHEDULES") or os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "schedules.json")
    if not os.path.exists(path):
        return False
    try:
        with open(path) as f:
            sel = json.load(f)
        _RAGGED_CHUNK = int(sel.get("ragged_chunk_tiles", 0))
        for km, bodies in sel.get("ragged_prefetch", {}).items():
            K, M = (int(v) for v in km.split("x"))
            for body, on in enumerate(bodies):
                # a choice this build cannot honour (no such class or body) keeps the default
                nat.load().transform_ragged_prefetch_select(K, M, body, int(on))
    except (OSError, ValueError, TypeError):
        _RAGGED_CHUNK = 0
    return nat.load().transform_load_schedule(path.encode()) == nat.TF_OK


def ragged_prefetch_select(K: int, M: int, body: int, prefetch: int):
    """Per-class tile pipelining of the ragged kernel for plans created afterwards: body 0
    forward, 1 inverse / adjoint, 2 adjoint with tap gradient; prefetch 0 off, 1 on (where
    that body has a prefetching form), -1 the compiled default."""
    nat.check("transform_ragged_prefetch_select",
              nat.load().transform_ragged_prefetch_select(K, M, body, prefetch))


def ragged_prefetch_selected(K: int, M: int, body: int) -> int:
    """The prefetch setting in effect for (K, M, body): 0 or 1."""
    v = ctypes.c_int32(0)
    nat.check("transform_ragged_prefetch_selected",
              nat.load().transform_ragged_prefetch_selected(K, M, body, ctypes.byref(v)))
    return int(v.value)


load_schedules()

__all__ = [
    "transform_forward", "transform_inverse", "transform_adjoint", "transform_inverse_adjoint",
    "transform_prepare", "workspace_size", "schedules", "select_schedule", "Transform",
    "InverseTransform", "forward", "inverse", "RaggedPlan", "bind_forward", "bind_adjoint",
    "selected_schedule", "transform_decimated", "transform_decimated_adjoint",
    "ragged_prefetch_select", "ragged_prefetch_selected",
]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _compute(c) -> int:
    return nat.COMPUTE[c] if isinstance(c, str) else int(c)


def _check_blocks(x: torch.Tensor, name: str, K: int, M: int) -> int:
    if not x.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if x.dtype != torch.complex64:
        raise TypeError(f"{name} must be complex64, got {x.dtype}")
    if x.dim() != 2 or x.shape[1] != K * M:
        raise ValueError(f"{name} must be [B, {K * M}], got {tuple(x.shape)}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x.shape[0]


def _tap_stride(taps: torch.Tensor, B: int, N: int, device) -> int:
    if taps.dtype != torch.float32 or not taps.is_contiguous() or taps.device != device:
        raise ValueError("taps must be contiguous float32 on the same device")
    if taps.shape == (N,):
        return 0
    if taps.shape == (B, N):
        return N
    raise ValueError(f"taps must be [{N}] or [{B}, {N}], got {tuple(taps.shape)}")


def workspace_size(B: int, K: int, M: int, tap_stride: int, compute="fp32", with_tapbar=False) -> int:
    return int(nat.load().transform_workspace_size(B, K, M, tap_stride, _compute(compute),
                                                   1 if with_tapbar else 0))


def _workspace(B, K, M, tap_stride, compute, with_tapbar, device):
    n = workspace_size(B, K, M, tap_stride, compute, with_tapbar)
    if n == 0:
        return None, 0
    return torch.empty(n, dtype=torch.uint8, device=device), n


def transform_prepare(K: int, M: int, compute="fp32"):
    nat.check("transform_prepare", nat.load().transform_prepare(K, M, _compute(compute)))


def transform_forward(coeffs: torch.Tensor, taps: torch.Tensor, K: int, M: int, *,
                      out: Optional[torch.Tensor] = None, compute="fp32") -> torch.Tensor:
    B = _check_blocks(coeffs, "coeffs", K, M)
    ts = _tap_stride(taps, B, K * M, coeffs.device)
    out = torch.empty_like(coeffs) if out is None else out
    _check_blocks(out, "samples", K, M)
    ws, wsb = _workspace(B, K, M, ts, compute, False, coeffs.device)
    nat.check("transform_forward", nat.load().transform_forward(
        _ptr(coeffs), _ptr(taps), _ptr(out), B, K, M, ts, _compute(compute), _ptr(ws), wsb,
        _stream(coeffs.device)))
    return out


def transform_inverse(samples: torch.Tensor, taps: torch.Tensor, K: int, M: int, *,
                      out: Optional[torch.Tensor] = None, status: Optional[torch.Tensor] = None,
                      compute="fp32") -> torch.Tensor:
    """`status` (int32 [1], zeroed by the caller) is set to 1 when a zero tap is met."""
    B = _check_blocks(samples, "samples", K, M)
    ts = _tap_stride(taps, B, K * M, samples.device)
    out = torch.empty_like(samples) if out is None else out
    _check_blocks(out, "coeffs", K, M)
    if status is not None and (status.dtype != torch.int32 or status.device != samples.device):
        raise ValueError("status must be an int32 tensor on the same device")
    ws, wsb = _workspace(B, K, M, ts, compute, False, samples.device)
    nat.check("transform_inverse", nat.load().transform_inverse(
        _ptr(samples), _ptr(taps), _ptr(out), B, K, M, ts, _compute(compute), _ptr(status),
        _ptr(ws), wsb, _stream(samples.device)))
    return out


def transform_adjoint(samples_bar: torch.Tensor, taps: torch.Tensor, K: int, M: int, *,
                      coeffs: Optional[torch.Tensor] = None, want_taps_bar: bool = False,
                      out: Optional[torch.Tensor] = None, taps_bar: Optional[torch.Tensor] = None,
                      compute="fp32") -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    B = _check_blocks(samples_bar, "samples_bar", K, M)
    N = K * M
    ts = _tap_stride(taps, B, N, samples_bar.device)
    out = torch.empty_like(samples_bar) if out is None else out
    _check_blocks(out, "coeffs_bar", K, M)
    tb = None
    if want_taps_bar or taps_bar is not None:
        if coeffs is None:
            raise ValueError("the tap gradient needs coeffs")
        _check_blocks(coeffs, "coeffs", K, M)
        tb = taps_bar if taps_bar is not None else torch.empty(
            (N,) if ts == 0 else (B, N), dtype=torch.float32, device=samples_bar.device)
    ws, wsb = _workspace(B, K, M, ts, compute, tb is not None, samples_bar.device)
    nat.check("transform_adjoint", nat.load().transform_adjoint(
        _ptr(samples_bar), _ptr(taps), _ptr(coeffs), _ptr(out), _ptr(tb), B, K, M, ts,
        _compute(compute), _ptr(ws), wsb, _stream(samples_bar.device)))
    return out, tb


def transform_inverse_adjoint(coeffs_bar: torch.Tensor, taps: torch.Tensor, K: int, M: int, *,
                              coeffs: Optional[torch.Tensor] = None, want_taps_bar: bool = False,
                              out: Optional[torch.Tensor] = None,
                              compute="fp32") -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    B = _check_blocks(coeffs_bar, "coeffs_bar", K, M)
    N = K * M
    ts = _tap_stride(taps, B, N, coeffs_bar.device)
    out = torch.empty_like(coeffs_bar) if out is None else out
    tb = None
    if want_taps_bar:
        if coeffs is None:
            raise ValueError("the tap gradient needs the inverse's output (coeffs)")
        _check_blocks(coeffs, "coeffs", K, M)
        tb = torch.empty((N,) if ts == 0 else (B, N), dtype=torch.float32, device=coeffs_bar.device)
    ws, wsb = _workspace(B, K, M, ts, compute, tb is not None, coeffs_bar.device)
    nat.check("transform_inverse_adjoint", nat.load().transform_inverse_adjoint(
        _ptr(coeffs_bar), _ptr(taps), _ptr(coeffs), _ptr(out), _ptr(tb), B, K, M, ts,
        _compute(compute), _ptr(ws), wsb, _stream(coeffs_bar.device)))
    return out, tb


# ------------------------------------------------------------------ decimated operator (eq. (7))
def transform_decimated(coeffs: torch.Tensor, taps: torch.Tensor, K: int, M: int, *,
                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[b, q] = sum_n taps_n S[b, n] e^{+j 2 pi n q / K}, q < K (eq. (7))."""
    B = _check_blocks(coeffs, "coeffs", K, M)
    ts = _tap_stride(taps, B, K * M, coeffs.device)
    out = torch.empty((B, K), dtype=torch.complex64, device=coeffs.device) if out is None else out
    if out.shape != (B, K) or out.dtype != torch.complex64 or not out.is_contiguous():
        raise ValueError(f"out must be contiguous complex64 [{B}, {K}]")
    nat.check("transform_decimated", nat.load().transform_decimated(
        _ptr(coeffs), _ptr(taps), _ptr(out), B, K, M, ts, _stream(coeffs.device)))
    return out


def transform_decimated_adjoint(samples_bar: torch.Tensor, taps: torch.Tensor, K: int, M: int, *,
                                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Sbar[b, n] = taps_n sum_q ybar[b, q] e^{-j 2 pi n q / K}."""
    if samples_bar.dtype != torch.complex64 or samples_bar.dim() != 2 or samples_bar.shape[1] != K \
            or not samples_bar.is_contiguous():
        raise ValueError(f"samples_bar must be contiguous complex64 [B, {K}]")
    B = samples_bar.shape[0]
    N = K * M
    ts = _tap_stride(taps, B, N, samples_bar.device)
    out = torch.empty((B, N), dtype=torch.complex64, device=samples_bar.device) if out is None else out
    _check_blocks(out, "coeffs_bar", K, M)
    nat.check("transform_decimated_adjoint", nat.load().transform_decimated_adjoint(
        _ptr(samples_bar), _ptr(taps), _ptr(out), B, K, M, ts, _stream(samples_bar.device)))
    return out


# ------------------------------------------------------------------ pre-marshalled calls
class BoundCall:
    """A transform call with every argument validated and marshalled once.

    Calling it re-issues the same C-ABI call on the same tensors (kept alive by
    the object) on the stream that was current when it was bound; it is the
    low-overhead path for loops that launch the same transform repeatedly."""

    def __init__(self, fn_name: str, args: tuple, device, keep: tuple):
        self._fn = getattr(nat.load(), fn_name)
        self._name = fn_name
        # the stream current at bind time is the one every call launches on
        self._args = args + (_stream(device),)
        self._keep = keep                      # tensors the pointers refer to

    def __call__(self):
        rc = self._fn(*self._args)
        if rc:
            nat.check(self._name, rc)


def bind_forward(coeffs, taps, K, M, out, compute="fp32") -> BoundCall:
    B = _check_blocks(coeffs, "coeffs", K, M)
    _check_blocks(out, "samples", K, M)
    ts = _tap_stride(taps, B, K * M, coeffs.device)
    ws, wsb = _workspace(B, K, M, ts, compute, False, coeffs.device)
    return BoundCall("transform_forward", (_ptr(coeffs), _ptr(taps), _ptr(out), B, K, M, ts,
                                           _compute(compute), _ptr(ws), wsb),
                     coeffs.device, (coeffs, taps, out, ws))


def bind_adjoint(samples_bar, taps, K, M, out, coeffs=None, taps_bar=None, compute="fp32") -> BoundCall:
    B = _check_blocks(samples_bar, "samples_bar", K, M)
    _check_blocks(out, "coeffs_bar", K, M)
    ts = _tap_stride(taps, B, K * M, samples_bar.device)
    if taps_bar is not None and coeffs is None:
        raise ValueError("the tap gradient needs coeffs")
    ws, wsb = _workspace(B, K, M, ts, compute, taps_bar is not None, samples_bar.device)
    return BoundCall("transform_adjoint", (_ptr(samples_bar), _ptr(taps), _ptr(coeffs), _ptr(out),
                                           _ptr(taps_bar), B, K, M, ts, _compute(compute),
                                           _ptr(ws), wsb),
                     samples_bar.device, (samples_bar, taps, coeffs, out, taps_bar, ws))


# ------------------------------------------------------------------ schedules
def schedules(K: int, M: int):
    import json
    lib = nat.load()
    out = []
    buf = ctypes.create_string_buffer(512)
    for i in range(lib.transform_schedule_count(K, M)):
        nat.check("transform_schedule_describe", lib.transform_schedule_describe(K, M, i, buf, 512))
        out.append(json.loads(buf.value.decode()))
    return out


def selected_schedule(K: int, M: int):
    """(index, grid cap, description) of the schedule currently used for (K, M)."""
    i, c = ctypes.c_int32(), ctypes.c_int32()
    nat.check("transform_schedule_selected", nat.load().transform_schedule_selected(
        K, M, ctypes.byref(i), ctypes.byref(c)))
    return i.value, c.value, schedules(K, M)[i.value]


def select_schedule(K: int, M: int, idx: int, grid_cap: int = 0):
    nat.check("transform_schedule_select", nat.load().transform_schedule_select(K, M, idx, grid_cap))


# ------------------------------------------------------------------ autograd
class Transform(torch.autograd.Function):
    """y = T_taps(S); gradients through the adjoint kernel (PyTorch's convention:
    grad_S = T^H grad_y, grad_taps = Re(conj(S) . W))."""

    @staticmethod
    def forward(ctx, S, taps, K, M):
        ctx.K, ctx.M = K, M
        ctx.save_for_backward(S, taps)
        return transform_forward(S.contiguous(), taps.contiguous(), K, M)

    @staticmethod
    def backward(ctx, gy):
        S, taps = ctx.saved_tensors
        need_taps = ctx.needs_input_grad[1]
        gS, gt = transform_adjoint(gy.contiguous(), taps, ctx.K, ctx.M,
                                   coeffs=S if need_taps else None, want_taps_bar=need_taps)
        return (gS if ctx.needs_input_grad[0] else None), gt, None, None


class InverseTransform(torch.autograd.Function):
    """S = T_taps^{-1}(y); gradients through the inverse's adjoint kernel."""

    @staticmethod
    def forward(ctx, y, taps, K, M):
        ctx.K, ctx.M = K, M
        S = transform_inverse(y.contiguous(), taps.contiguous(), K, M)
        ctx.save_for_backward(taps, S)
        return S

    @staticmethod
    def backward(ctx, gS):
        taps, S = ctx.saved_tensors
        need_taps = ctx.needs_input_grad[1]
        gy, gt = transform_inverse_adjoint(gS.contiguous(), taps, ctx.K, ctx.M,
                                           coeffs=S if need_taps else None, want_taps_bar=need_taps)
        return (gy if ctx.needs_input_grad[0] else None), gt, None, None


def forward(S, taps, K, M):
    return Transform.apply(S, taps, K, M)


def inverse(y, taps, K, M):
    return InverseTransform.apply(y, taps, K, M)


# ------------------------------------------------------------------ ragged batches
class RaggedPlan:
    """Plan for a batch of blocks with their own (K, M), run as one grouped launch per call.

    `K`, `M`, `x_off`, `tap_off` are host arrays (one entry per block; offsets in
    elements of the flat complex / tap arrays); `total_points` is the length of
    the flat complex arrays.  The plan owns its device tables and HIP graphs.
    """

    DIRECTIONS = {"forward": 0, "inverse": 1, "adjoint": 2}

    def __init__(self, K, M, x_off, tap_off, total_points: int, chunk_tiles: Optional[int] = None):
        import numpy as np
        K = np.ascontiguousarray(K, dtype=np.int32)
        M = np.ascontiguousarray(M, dtype=np.int32)
        xo = np.ascontiguousarray(x_off, dtype=np.int64)
        to = np.ascontiguousarray(tap_off, dtype=np.int64)
        if not (K.shape == M.shape == xo.shape == to.shape):
            raise ValueError("K, M, x_off, tap_off must have one entry per block")
        self.total_points = int(total_points)
        self.nblocks = int(K.size)
        self._lib = nat.load()
        if chunk_tiles is None:
            chunk_tiles = _RAGGED_CHUNK
        h = ctypes.c_void_p()
        nat.check("transform_ragged_plan_create", self._lib.transform_ragged_plan_create_ex(
            K.ctypes.data_as(ctypes.c_void_p), M.ctypes.data_as(ctypes.c_void_p),
            xo.ctypes.data_as(ctypes.c_void_p), to.ctypes.data_as(ctypes.c_void_p),
            self.nblocks, self.total_points, int(chunk_tiles), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.transform_ragged_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def execute(self, direction: str, x: torch.Tensor, taps: torch.Tensor, *,
                out: Optional[torch.Tensor] = None, aux: Optional[torch.Tensor] = None,
                want_taps_bar: bool = False, status: Optional[torch.Tensor] = None,
                use_graph: bool = True):
        """direction: "forward" (x = S), "inverse" (x = y), "adjoint" (x = ybar; with
        want_taps_bar, aux = S and the per-block tap gradient is returned laid out
        like the coefficients)."""
        d = self.DIRECTIONS[direction]
        if x.dtype != torch.complex64 or x.dim() != 1 or x.numel() != self.total_points:
            raise ValueError(f"x must be complex64 [{self.total_points}]")
        if not x.is_contiguous() or not x.is_cuda:
            raise ValueError("x must be a contiguous GPU tensor")
        if taps.dtype != torch.float32 or not taps.is_contiguous() or taps.device != x.device:
            raise ValueError("taps must be contiguous float32 on the same device")
        out = torch.empty_like(x) if out is None else out
        tb = None
        if want_taps_bar:
            if d != 2 or aux is None:
                raise ValueError("the tap gradient is an adjoint output and needs aux = S")
            tb = torch.empty(self.total_points, dtype=torch.float32, device=x.device)
        nat.check("transform_ragged_execute", self._lib.transform_ragged_execute(
            self._h, d, _ptr(x), _ptr(taps), _ptr(out), _ptr(aux), _ptr(tb), _ptr(status),
            1 if use_graph else 0, _stream(x.device)))
        return (out, tb) if want_taps_bar else out

    def bind(self, direction: str, x: torch.Tensor, taps: torch.Tensor, out: torch.Tensor, *,
             aux: Optional[torch.Tensor] = None, taps_bar: Optional[torch.Tensor] = None,
             use_graph: bool = True) -> BoundCall:
        """One execution with its arguments checked and marshalled once (see BoundCall)."""
        d = self.DIRECTIONS[direction]
        for t, name in ((x, "x"), (out, "out")):
            if t.dtype != torch.complex64 or t.numel() != self.total_points or not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous complex64 [{self.total_points}]")
        if taps.dtype != torch.float32 or not taps.is_contiguous():
            raise ValueError("taps must be contiguous float32")
        if taps_bar is not None and (d != 2 or aux is None):
            raise ValueError("the tap gradient is an adjoint output and needs aux = S")
        return BoundCall("transform_ragged_execute",
                         (self._h, d, _ptr(x), _ptr(taps), _ptr(out), _ptr(aux), _ptr(taps_bar), None,
                          1 if use_graph else 0), x.device, (self, x, taps, out, aux, taps_bar))
