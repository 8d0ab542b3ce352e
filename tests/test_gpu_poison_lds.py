"""The LDS-poisoning test build (libblocktransform_poison.so: every fused, ragged and
decimated kernel fills its LDS with NaN on entry) at the benchmark's launch shapes, against
the FP64 oracle.  A read of LDS that no thread of the launch has written -- a missing store,
or a barrier in the wrong place on the first block group -- would make outputs NaN."""
import ctypes
import os

import numpy as np
import pytest

from oracle import fftref as F
from oracle import oracle as O
from paper_1604_06236_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5
PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1604_06236_amd")
POISON_LIB = os.path.join(PKG, "libblocktransform_poison.so")


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a, np.complex128) - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    assert os.path.exists(POISON_LIB), "build with poison=True first"
    lib = ctypes.CDLL(POISON_LIB)
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.transform_forward.argtypes = [vp, vp, vp, i64, i32, i32, i64, i32, vp, sz, vp]
    lib.transform_adjoint.argtypes = [vp, vp, vp, vp, vp, i64, i32, i32, i64, i32, vp, sz, vp]
    lib.transform_decimated.argtypes = [vp, vp, vp, i64, i32, i32, i64, vp]
    lib.transform_ragged_plan_create_ex.argtypes = [vp, vp, vp, vp, i64, i64, i32, ctypes.POINTER(vp)]
    lib.transform_ragged_execute.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, i32, vp]
    lib.transform_ragged_plan_destroy.argtypes = [vp]
    lib.transform_load_schedule.argtypes = [ctypes.c_char_p]
    # the same schedule choices as the benchmark
    assert lib.transform_load_schedule(os.path.join(PKG, "schedules.json").encode()) == 0
    return torch, lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _s(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_poisoned_fused_at_benchmark_shapes(env):
    torch, lib = env
    for cfg in ("plain_gpu", "precision", "differentiation"):
        c = W.CONFIGS[cfg]
        S, taps = W.make_uniform(cfg)
        B, N = S.shape
        yb = W.cn01(np.random.default_rng(3), (B, N)).astype(np.complex64)
        print(f"case poison fused {cfg}", flush=True)
        dS, dt, dyb = (torch.from_numpy(x).cuda() for x in (S, taps, yb))
        y, sb = torch.empty_like(dS), torch.empty_like(dS)
        assert lib.transform_forward(_p(dS), _p(dt), _p(y), B, c.K, c.M, 0, 0, None, 0, _s(torch)) == 0
        assert lib.transform_adjoint(_p(dyb), _p(dt), None, _p(sb), None, B, c.K, c.M, 0, 0, None, 0,
                                     _s(torch)) == 0
        torch.cuda.synchronize()
        yh, sbh = y.cpu().numpy(), sb.cpu().numpy()
        assert np.all(np.isfinite(yh)) and np.all(np.isfinite(sbh))
        assert rel(yh, F.forward(S, taps)) < TOL
        assert rel(sbh, F.adjoint(yb, taps)[0]) < TOL
        idx = np.array([0, B // 2, B - 1])
        assert rel(yh[idx], O.forward(S[idx], taps)) < TOL


def test_poisoned_half_lds_schedules(env):
    """Every (1024, M) half-block exchange schedule with its LDS prefilled with NaN: a missing
    barrier between an exchange round's writes and reads would let NaN through."""
    torch, lib = env
    from paper_1604_06236_amd import transform as T
    lib.transform_schedule_select.argtypes = [ctypes.c_int32] * 4
    for M in (3, 9, 15):
        K, B = 1024, 37
        idx = [i for i, d in enumerate(T.schedules(K, M)) if d.get("half_lds")]
        assert idx, M
        rng = np.random.default_rng(M)
        S = W.cn01(rng, (B, K * M)).astype(np.complex64)
        taps = W.rc_taps(K * M, 0.3).astype(np.float32)
        yb = W.cn01(rng, (B, K * M)).astype(np.complex64)
        dS, dt, dyb = (torch.from_numpy(x).cuda() for x in (S, taps, yb))
        y, sb = torch.empty_like(dS), torch.empty_like(dS)
        print(f"case poison half K={K} M={M} schedule={idx[0]}", flush=True)
        try:
            assert lib.transform_schedule_select(K, M, idx[0], 5) == 0      # several blocks per workgroup
            assert lib.transform_forward(_p(dS), _p(dt), _p(y), B, K, M, 0, 0, None, 0, _s(torch)) == 0
            assert lib.transform_adjoint(_p(dyb), _p(dt), None, _p(sb), None, B, K, M, 0, 0, None, 0,
                                         _s(torch)) == 0
            torch.cuda.synchronize()
        finally:
            lib.transform_load_schedule(os.path.join(PKG, "schedules.json").encode())
        yh, sbh = y.cpu().numpy(), sb.cpu().numpy()
        assert np.all(np.isfinite(yh)) and np.all(np.isfinite(sbh))
        assert rel(yh, F.forward(S, taps)) < TOL
        assert rel(sbh, F.adjoint(yb, taps)[0]) < TOL


def test_poisoned_decimated(env):
    torch, lib = env
    c = W.CONFIGS["plain_gpu"]
    S, taps = W.make_uniform("plain_gpu")
    B = S.shape[0]
    dS, dt = torch.from_numpy(S).cuda(), torch.from_numpy(taps).cuda()
    d = torch.empty((B, c.K), dtype=torch.complex64, device="cuda")
    assert lib.transform_decimated(_p(dS), _p(dt), _p(d), B, c.K, c.M, 0, _s(torch)) == 0
    torch.cuda.synchronize()
    dh = d.cpu().numpy()
    assert np.all(np.isfinite(dh))
    idx = np.array([0, 1, 2047, 4095])
    assert rel(dh[idx], O.decimated(S[idx], taps, c.K)) < TOL


def test_poisoned_ragged_full_batch(env):
    torch, lib = env
    lay, S, taps = W.make_ragged("ragged")
    print("case poison ragged", flush=True)
    K = np.ascontiguousarray(lay.K, np.int32)
    M = np.ascontiguousarray(lay.M, np.int32)
    xo = np.ascontiguousarray(lay.x_off, np.int64)
    to = np.ascontiguousarray(lay.tap_off, np.int64)
    h = ctypes.c_void_p()
    assert lib.transform_ragged_plan_create_ex(K.ctypes.data_as(ctypes.c_void_p), M.ctypes.data_as(ctypes.c_void_p),
                                               xo.ctypes.data_as(ctypes.c_void_p), to.ctypes.data_as(ctypes.c_void_p),
                                               K.size, lay.total, 4, ctypes.byref(h)) == 0
    try:
        dS, dt = torch.from_numpy(S).cuda(), torch.from_numpy(taps).cuda()
        y = torch.empty_like(dS)
        assert lib.transform_ragged_execute(h, 0, _p(dS), _p(dt), _p(y), None, None, None, 1, _s(torch)) == 0
        torch.cuda.synchronize()
        yh = y.cpu().numpy()
        assert np.all(np.isfinite(yh))
        assert rel(yh, F.forward_ragged(lay.N, lay.x_off, lay.tap_off, S, taps)) < TOL
    finally:
        lib.transform_ragged_plan_destroy(h)
