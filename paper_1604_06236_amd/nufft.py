"""Python binding of the non-iterative type-5 / type-4 NFFT methods and the exact
type-1 / type-2 sums (argument marshalling only; every step runs in the HIP
library, which must be built).

Shapes: t float64 [B, P] (instants, read modulo 1), complex data complex64
[B, P] (or [B, R] for a type-1 output), all contiguous on the GPU.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import torch

from . import _native as nat


def _ptr(x: Optional[torch.Tensor]):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(x: torch.Tensor, name: str, dtype, shape=None):
    if not x.is_cuda or not x.is_contiguous() or x.dtype != dtype or x.dim() != 2:
        raise ValueError(f"{name} must be a contiguous 2-D {dtype} GPU tensor")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")


def damping_for(mu: float, eta: int, P: int) -> float:
    """Damping a that gives the truncation ratio mu of eq. (49),
    mu = exp(-2 pi (eta P - 1) a) / (eta P - 1)."""
    n = eta * P - 1
    return -math.log(mu * n) / (2.0 * math.pi * n)


NUFFT_REFINE = 1
NUFFT_GRIDDING = 2


def nufft_workspace_size(B: int, P: int, eta: int, flags: int = 0) -> int:
    return int(nat.load().nufft_workspace_size_ex(B, P, eta, flags))


def nufft_solve(kind: int, t: torch.Tensor, x: torch.Tensor, eta: int, a: float, *,
                refine: bool = False, gridding: bool = False, out: Optional[torch.Tensor] = None,
                workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """kind 5: coefficients from samples (eq. (48)); kind 4: amplitudes from the
    spectrum (eq. (47)).  `refine`: the refined method of Sec. 5; `gridding`: the
    non-uniform sums by gridding NFFTs instead of exact sums."""
    _check(t, "t", torch.float64)
    B, P = t.shape
    _check(x, "input", torch.complex64, (B, P))
    out = torch.empty_like(x) if out is None else out
    _check(out, "out", torch.complex64, (B, P))
    flags = (NUFFT_REFINE if refine else 0) | (NUFFT_GRIDDING if gridding else 0)
    need = nufft_workspace_size(B, P, eta, flags)
    if need == 0:
        nat.check("nufft_solve", nat.TF_EUNSUPPORTED)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    if workspace.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    nat.check("nufft_solve", nat.load().nufft_solve(
        int(kind), flags, _ptr(t), _ptr(x), _ptr(out), B, P, eta, float(a), _ptr(workspace),
        workspace.numel(), _stream(x.device)))
    return out


def nufft_setup(t: torch.Tensor, eta: int, a: float, *, gridding: bool = False,
                workspace: Optional[torch.Tensor] = None, refine: bool = False) -> torch.Tensor:
    """The part of both methods that depends on the instants only (filters, kernel
    samples eq. (28)-(29), Lagrange coefficients eq. (43), derivative samples
    eq. (16)), into a workspace that nufft_apply reuses; returns the workspace.
    `refine` only sizes the workspace for refined applications."""
    _check(t, "t", torch.float64)
    B, P = t.shape
    flags = (NUFFT_REFINE if refine else 0) | (NUFFT_GRIDDING if gridding else 0)
    need = nufft_workspace_size(B, P, eta, flags)
    if need == 0:
        nat.check("nufft_setup", nat.TF_EUNSUPPORTED)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=t.device)
    if workspace.numel() < need:
        raise ValueError(f"workspace needs {need} bytes")
    nat.check("nufft_setup", nat.load().nufft_setup(
        NUFFT_GRIDDING if gridding else 0, _ptr(t), B, P, eta, float(a), _ptr(workspace), workspace.numel(),
        _stream(t.device)))
    return workspace


def nufft_apply(kind: int, t: torch.Tensor, x: torch.Tensor, eta: int, a: float, workspace: torch.Tensor, *,
                refine: bool = False, gridding: bool = False,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """nufft_solve from a workspace prepared by nufft_setup for the same t, eta, a."""
    _check(t, "t", torch.float64)
    B, P = t.shape
    _check(x, "input", torch.complex64, (B, P))
    out = torch.empty_like(x) if out is None else out
    _check(out, "out", torch.complex64, (B, P))
    flags = (NUFFT_REFINE if refine else 0) | (NUFFT_GRIDDING if gridding else 0)
    nat.check("nufft_apply", nat.load().nufft_apply(
        int(kind), flags, _ptr(t), _ptr(x), _ptr(out), B, P, eta, float(a), _ptr(workspace),
        workspace.numel(), _stream(x.device)))
    return out


def nufft_type5(t: torch.Tensor, samples: torch.Tensor, eta: int, a: float, *,
                out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                refine: bool = False, gridding: bool = False):
    """Coefficients S [B, P] with sum_p S_p e^{j 2 pi p t_q} = samples_q (eq. (48))."""
    return nufft_solve(5, t, samples, eta, a, refine=refine, gridding=gridding, out=out, workspace=workspace)


def nufft_type4(t: torch.Tensor, spectrum: torch.Tensor, eta: int, a: float, *,
                out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                refine: bool = False, gridding: bool = False):
    """Amplitudes a [B, P] with sum_q a_q e^{-j 2 pi r t_q} = spectrum_r, r < P (eq. (47))."""
    return nufft_solve(4, t, spectrum, eta, a, refine=refine, gridding=gridding, out=out, workspace=workspace)


def nudft_type1(t: torch.Tensor, amp: Optional[torch.Tensor], R: int, *,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[b, r] = sum_q amp[b, q] e^{-j 2 pi r t[b, q]}, r < R (eq. (32)); amp None = ones."""
    _check(t, "t", torch.float64)
    B, Q = t.shape
    if amp is not None:
        _check(amp, "amp", torch.complex64, (B, Q))
    out = torch.empty((B, R), dtype=torch.complex64, device=t.device) if out is None else out
    _check(out, "out", torch.complex64, (B, R))
    nat.check("nudft_type1", nat.load().nudft_type1(_ptr(t), _ptr(amp), _ptr(out), B, Q, R,
                                                    _stream(t.device)))
    return out


def nudft_type2(t: torch.Tensor, coeffs: torch.Tensor, *,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[b, q] = sum_p coeffs[b, p] e^{+j 2 pi p t[b, q]} (eq. (34))."""
    _check(t, "t", torch.float64)
    B, Q = t.shape
    if coeffs.dim() != 2 or coeffs.shape[0] != B:
        raise ValueError("coeffs must be [B, P]")
    _check(coeffs, "coeffs", torch.complex64)
    P = coeffs.shape[1]
    out = torch.empty((B, Q), dtype=torch.complex64, device=t.device) if out is None else out
    _check(out, "out", torch.complex64, (B, Q))
    nat.check("nudft_type2", nat.load().nudft_type2(_ptr(t), _ptr(coeffs), _ptr(out), B, P, Q,
                                                    _stream(t.device)))
    return out


def nfft_type1(t: torch.Tensor, amp: Optional[torch.Tensor], R: int, *,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gridding type-1 NFFT (Gaussian window, oversampling 2): approximates nudft_type1."""
    _check(t, "t", torch.float64)
    B, Q = t.shape
    if amp is not None:
        _check(amp, "amp", torch.complex64, (B, Q))
    out = torch.empty((B, R), dtype=torch.complex64, device=t.device) if out is None else out
    _check(out, "out", torch.complex64, (B, R))
    need = int(nat.load().nfft_workspace_size(B, R))
    if need == 0:
        nat.check("nfft_type1", nat.TF_EUNSUPPORTED)
    ws = torch.empty(need, dtype=torch.uint8, device=t.device)
    nat.check("nfft_type1", nat.load().nfft_type1(_ptr(t), _ptr(amp), _ptr(out), B, Q, R, _ptr(ws), need,
                                                  _stream(t.device)))
    return out


def nfft_type2(t: torch.Tensor, coeffs: torch.Tensor, *,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gridding type-2 NFFT (Gaussian window, oversampling 2): approximates nudft_type2."""
    _check(t, "t", torch.float64)
    B, Q = t.shape
    _check(coeffs, "coeffs", torch.complex64)
    if coeffs.shape[0] != B:
        raise ValueError("coeffs must be [B, P]")
    P = coeffs.shape[1]
    out = torch.empty((B, Q), dtype=torch.complex64, device=t.device) if out is None else out
    _check(out, "out", torch.complex64, (B, Q))
    need = int(nat.load().nfft_workspace_size(B, P))
    if need == 0:
        nat.check("nfft_type2", nat.TF_EUNSUPPORTED)
    ws = torch.empty(need, dtype=torch.uint8, device=t.device)
    nat.check("nfft_type2", nat.load().nfft_type2(_ptr(t), _ptr(coeffs), _ptr(out), B, P, Q, _ptr(ws), need,
                                                  _stream(t.device)))
    return out
