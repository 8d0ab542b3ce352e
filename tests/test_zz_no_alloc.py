"""The allocation-free adjoint (transform_adjoint_noalloc), called through the C ABI, against
the existing entry point transform_adjoint on the same inputs, and against the FP64 oracle:
two calls in a row, the second with a smaller input, each relative L2 <= 1e-5."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_06236_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.complex128 if np.iscomplexobj(a) else np.float64)
    b = np.asarray(b, np.complex128 if np.iscomplexobj(b) else np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1604_06236_amd import _native as nat
    from paper_1604_06236_amd import transform as T
    return torch, nat, T, nat.load()


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _case(env, B, K, M, shared, tapgrad, seed):
    torch, nat, T, lib = env
    N = K * M
    rng = np.random.default_rng(seed)
    S = W.cn01(rng, (B, N)).astype(np.complex64)
    yb = W.cn01(rng, (B, N)).astype(np.complex64)
    taps = (W.rc_taps(N, 0.3) if shared else
            np.stack([W.rc_taps(N, a) for a in rng.uniform(0.1, 0.9, B)])).astype(np.float32)
    dS, dyb, dt = (torch.from_numpy(x).cuda() for x in (S, yb, taps))
    sb = torch.empty_like(dS)
    tb = torch.empty((N,) if shared else (B, N), dtype=torch.float32, device="cuda") if tapgrad else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    print(f"case noalloc B={B} K={K} M={M} shared={shared} tapgrad={tapgrad}", flush=True)
    rc = lib.transform_adjoint_noalloc(_p(dyb), _p(dt), _p(dS) if tapgrad else None, _p(sb), _p(tb),
                                       B, K, M, 0 if shared else N, stream)
    assert rc == nat.TF_OK, nat.status_string(rc)
    torch.cuda.synchronize()
    ref_sb, ref_tb = T.transform_adjoint(dyb, dt, K, M, coeffs=dS if tapgrad else None,
                                         want_taps_bar=tapgrad)
    torch.cuda.synchronize()
    got_sb = sb.cpu().numpy()
    assert rel(got_sb, ref_sb.cpu().numpy()) < TOL
    o_sb, o_tb = O.adjoint(yb, taps, S if tapgrad else None)
    assert rel(got_sb, o_sb) < TOL
    if tapgrad:
        got_tb = tb.cpu().numpy()
        assert rel(got_tb, ref_tb.cpu().numpy()) < TOL
        assert rel(got_tb, o_tb) < TOL


def test_scratch_size(env):
    _, _, _, lib = env
    assert lib.transform_noalloc_scratch_bytes() == 16 << 20


def test_two_calls_second_smaller(env):
    """The shared tap gradient (the case that uses the scratch array): a large call, then a
    smaller one on the same array."""
    _case(env, 2048, 256, 9, shared=True, tapgrad=True, seed=1)
    _case(env, 37, 128, 15, shared=True, tapgrad=True, seed=2)


def test_capped_grid_and_other_modes(env):
    """A block size whose partial rows cap the grid (K=1024, M=15), then per-block taps and a
    plain adjoint (no scratch needed), each followed by a smaller call."""
    _case(env, 600, 1024, 15, shared=True, tapgrad=True, seed=3)
    _case(env, 5, 64, 3, shared=True, tapgrad=True, seed=4)
    _case(env, 64, 256, 9, shared=False, tapgrad=True, seed=5)
    _case(env, 9, 16, 5, shared=True, tapgrad=False, seed=6)


def test_errors_before_launch(env):
    torch, nat, _, lib = env
    x = torch.zeros((4, 80), dtype=torch.complex64, device="cuda")
    t = torch.ones(80, device="cuda")
    assert lib.transform_adjoint_noalloc(_p(x), _p(t), None, _p(x), None, 4, 16, 5, 0, None) == nat.TF_EINVAL
    assert lib.transform_adjoint_noalloc(_p(x), _p(t), None, _p(torch.empty_like(x)), None, 4, 3, 5, 0,
                                         None) == nat.TF_EUNSUPPORTED
    # the tap gradient needs the coefficients
    assert lib.transform_adjoint_noalloc(_p(x), _p(t), None, _p(torch.empty_like(x)), _p(t.clone()), 4, 16,
                                         5, 0, None) == nat.TF_EINVAL
