"""Split-precision MFMA GEMM-DFT path against the FP64 oracle, to its stated bound.

Bound.  Each real operand x is stored as hi + lo in a 16-bit format with p
significant bits (BF16: p = 8, FP16: p = 11), so |x - hi - lo| <= 2^-2p |x|; a real
product formed from three of the four partial products is off by at most about
3 * 2^-2p of |a b|.  A length-L DFT stage turns per-term relative errors d into an
output error of at most d * sqrt(L) relative to the output norm (all weights have
modulus 1), so the three stages (L = 16, KS, KS) add up to
    3 * 2^-2p * (4 + 2 sqrt(KS))
plus FP32 rounding of the accumulations and twiddles (a few 1e-7).  For KS = 32:
BF16 -> 1.75e-4, FP16 -> 2.7e-6; the tests allow 2e-4 and 3e-6 relative L2.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_06236_amd import workloads as W

pytestmark = pytest.mark.gpu

BOUND = {"split_bf16": 2e-4, "split_fp16": 3e-6}


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a, np.complex128) - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_1604_06236_amd import transform
    return transform


@pytest.mark.parametrize("compute", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("K,M", [(1024, 15), (256, 9), (256, 1), (1024, 16), (256, 5)])
@pytest.mark.parametrize("shared", [True, False])
def test_split_forward_adjoint(T, compute, K, M, shared):
    B = 6
    N = K * M
    print(f"case split {compute} K={K} M={M} shared={shared}", flush=True)
    rng = np.random.default_rng(K + M)
    S = W.cn01(rng, (B, N)).astype(np.complex64)
    taps = (W.rrc_taps(N, 0.1) if shared else
            np.stack([W.rc_taps(N, a) for a in rng.uniform(0.1, 0.9, B)])).astype(np.float32)
    y = _host(T.transform_forward(_dev(S), _dev(taps), K, M, compute=compute))
    y_ref = O.forward(S, taps)
    e_f = rel_l2(y, y_ref)
    yb = W.cn01(rng, (B, N)).astype(np.complex64)
    sb, _ = T.transform_adjoint(_dev(yb), _dev(taps), K, M, compute=compute)
    sb_ref, _ = O.adjoint(yb, taps)
    e_a = rel_l2(_host(sb), sb_ref)
    print(f"  rel-L2 forward {e_f:.2e} adjoint {e_a:.2e} (bound {BOUND[compute]:.1e})", flush=True)
    assert e_f < BOUND[compute] and e_a < BOUND[compute]
    # the split is doing its job: far better than one 16-bit rounding (2^-p)
    assert e_f < 0.05 * 2.0 ** -(8 if compute == "split_bf16" else 11)


def test_split_precision_config_full_size(T):
    """The full precision workload (2048 blocks, K=1024, M=15): sampled blocks
    against the oracle for both formats, and agreement with the FP32 FFT path."""
    S, taps = W.make_uniform("precision")
    K, M = 1024, 15
    dS, dt = _dev(S), _dev(taps)
    y32 = _host(T.transform_forward(dS, dt, K, M))
    idx = np.array([0, 517, 1023, 2047])
    ref = O.forward(S[idx], taps)
    yb = W.cn01(np.random.default_rng(31), S.shape).astype(np.complex64)
    dyb = _dev(yb)
    sb32, _ = T.transform_adjoint(dyb, dt, K, M)
    sb32 = _host(sb32)
    sb_ref, _ = O.adjoint(yb[idx], taps)
    for compute in ("split_bf16", "split_fp16"):
        print(f"case split full {compute}", flush=True)
        y = _host(T.transform_forward(dS, dt, K, M, compute=compute))
        assert rel_l2(y[idx], ref) < BOUND[compute]
        assert rel_l2(y, y32.astype(np.complex128)) < BOUND[compute] + 1e-6
        # the adjoint over the same persistent launch (eight blocks per workgroup)
        sb, _ = T.transform_adjoint(dyb, dt, K, M, compute=compute)
        sb = _host(sb)
        assert rel_l2(sb[idx], sb_ref) < BOUND[compute]
        assert rel_l2(sb, sb32.astype(np.complex128)) < BOUND[compute] + 1e-6


def test_split_rejects_unsupported(T):
    from paper_1604_06236_amd._native import TransformError
    x = _dev(np.zeros((1, 128 * 3), np.complex64))
    with pytest.raises(TransformError):
        T.transform_forward(x, _dev(np.ones(384, np.float32)), 128, 3, compute="split_bf16")
