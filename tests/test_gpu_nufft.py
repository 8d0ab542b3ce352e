"""GPU type-1 / type-2 sums and the type-5 / type-4 methods against the FP64
oracle (oracle/lagrange.py) and Gaussian elimination.

Tolerances.  The sums use exact fixed-point phases, FP32 terms and FP64
accumulation: relative error a few FP32 ulps (bound 2e-6 here).  The methods run
every regular-grid step in FP32; eq. (43) multiplies the FP32 rounding of the
kernel samples by up to amp = exp(2 pi a (P - 1)) (the damping compensation),
so the GPU-vs-oracle tolerance is 4e-6 * amp (a few FP32 ulps times the
log2 P depth of the transforms, times amp).
"""
import math

import numpy as np
import pytest

from oracle import lagrange as L
from paper_1604_06236_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1604_06236_amd import nufft as NU
    from paper_1604_06236_amd import _native as nat
    return torch, NU, nat


def cn(rng, shape):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)).astype(np.complex64)


def inst(B, P, seed):
    rng = np.random.default_rng(seed)
    return np.stack([W.jittered_instants(rng, P) for _ in range(B)])


def dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("Q,R,unit", [(64, 384, False), (100, 1000, False), (1, 7, False), (256, 4096, True),
                                      (1024, 1024, False), (20, 640, False), (300, 1024, True),
                                      (2500, 1000, False), (3, 65, True)])
def test_type1_sum_matches_oracle(env, Q, R, unit):
    torch, NU, _ = env
    B = 3
    t = inst(B, Q, Q + R)
    rng = np.random.default_rng(R)
    amp = None if unit else cn(rng, (B, Q))
    out = NU.nudft_type1(dev(torch, t), None if unit else dev(torch, amp), R).cpu().numpy()
    for b in range(B):
        ref = L.type1(t[b], np.ones(Q) if unit else amp[b], R)
        # FP64 tables and FP64 matrix-core accumulation: only the FP32 input and output
        # roundings remain (R is padded to a multiple of 64 inside)
        assert L.rel_err(out[b], ref) < 5e-7


def test_type1_sum_wide_matrix_core_tiles(env):
    """A batch large enough for the three-column-tile launch, a chunk tail (Q not a
    multiple of 16) and a partial last column tile (R / 64 = 100 columns)."""
    torch, NU, _ = env
    B, Q, R = 320, 37, 6400
    t = inst(B, Q, 11)
    amp = cn(np.random.default_rng(12), (B, Q))
    out = NU.nudft_type1(dev(torch, t), dev(torch, amp), R).cpu().numpy()
    for b in list(range(0, B, 29)) + [B - 1]:
        assert L.rel_err(out[b], L.type1(t[b], amp[b], R)) < 5e-7


@pytest.mark.parametrize("P,Q", [(64, 64), (64, 77), (1024, 300), (5, 1), (192, 50), (100, 130), (2000, 90),
                                 (65, 3)])
def test_type2_sum_matches_oracle(env, P, Q):
    torch, NU, _ = env
    B = 2
    t = inst(B, Q, 7 * P + Q)
    c = cn(np.random.default_rng(P), (B, P))
    out = NU.nudft_type2(dev(torch, t), dev(torch, c)).cpu().numpy()
    for b in range(B):
        assert L.rel_err(out[b], L.type2(c[b], t[b])) < 5e-7


def test_sums_read_instants_modulo_one(env):
    torch, NU, _ = env
    t = inst(2, 64, 3)
    shifted = t + np.array([[3.0], [-2.0]])
    amp = cn(np.random.default_rng(4), (2, 64))
    a1 = NU.nudft_type1(dev(torch, t), dev(torch, amp), 256).cpu().numpy()
    a2 = NU.nudft_type1(dev(torch, shifted), dev(torch, amp), 256).cpu().numpy()
    assert L.rel_err(a2, a1) < 1e-6


def amp_of(a, P):
    return math.exp(2 * math.pi * a * (P - 1))


# The FP32 regular-grid steps serve a (P, eta, mu) when the amplified FP32 bound stays
# meaningful: 4e-6 * exp(2 pi a (P - 1)) <= 1e-3.  eta = 1 needs a large damping a for a
# small mu (eq. (49) with eta P - 1 = P - 1), so mu = 1e-7 at P = 64 amplifies FP32 rounding
# by 1.6e5 and is outside what the FP32 method can serve; mu = 1e-3 there amplifies by 16.
TOL_CAP = 1e-3


def method_tol(a, P):
    tol = 4e-6 * amp_of(a, P)
    assert tol <= TOL_CAP, f"(a={a}, P={P}) is outside what the FP32 method serves (tolerance {tol:.2g})"
    return tol


def test_fp32_service_range():
    """The cap rejects the eta = 1, mu = 1e-7 case and admits the cases tested below."""
    from paper_1604_06236_amd import nufft as NU
    with pytest.raises(AssertionError):
        method_tol(NU.damping_for(1e-7, 1, 64), 64)
    assert method_tol(NU.damping_for(1e-3, 1, 64), 64) < 1e-4


@pytest.mark.parametrize("P,eta,mu", [(16, 6, 1e-7), (64, 1, 1e-3), (64, 6, 1e-7), (256, 15, 1e-7),
                                      (1024, 6, 1e-7), (1024, 15, 1e-6),
                                      pytest.param(64, 1, 1e-7, marks=pytest.mark.skip(
                                          reason="eta = 1 at mu = 1e-7 amplifies FP32 rounding by "
                                                 "exp(2 pi a (P-1)) = 1.6e5: outside the FP32 method's range"))])
def test_methods_match_oracle(env, P, eta, mu):
    torch, NU, _ = env
    B = 3 if P < 1024 else 2
    a = NU.damping_for(mu, eta, P)
    t = inst(B, P, 11 * P + eta)
    rng = np.random.default_rng(P + eta)
    s = cn(rng, (B, P))
    A = cn(rng, (B, P))
    S_gpu = NU.nufft_type5(dev(torch, t), dev(torch, s), eta, a).cpu().numpy()
    a_gpu = NU.nufft_type4(dev(torch, t), dev(torch, A), eta, a).cpu().numpy()
    tol = method_tol(a, P)
    for b in range(B):
        st = L.Setup(t[b], eta, a)
        assert L.rel_err(S_gpu[b], L.type5_method(t[b], s[b], eta, a, st)) < tol
        assert L.rel_err(a_gpu[b], L.type4_method(t[b], A[b], eta, a, st)) < tol


def test_methods_solve_the_systems(env):
    """At P = 64, eta = 6 the GPU solutions agree with Gaussian elimination on
    eq. (48) / eq. (47) to the method's truncation error plus the FP32 bound."""
    torch, NU, _ = env
    P, eta, mu, B = 64, 6, 1e-7, 4
    a = NU.damping_for(mu, eta, P)
    t = inst(B, P, 99)
    rng = np.random.default_rng(5)
    s = cn(rng, (B, P))
    A = cn(rng, (B, P))
    S_gpu = NU.nufft_type5(dev(torch, t), dev(torch, s), eta, a).cpu().numpy()
    a_gpu = NU.nufft_type4(dev(torch, t), dev(torch, A), eta, a).cpu().numpy()
    for b in range(B):
        e5 = L.rel_err(L.type5_method(t[b], s[b], eta, a), L.ge_type5(t[b], s[b]))
        e4 = L.rel_err(L.type4_method(t[b], A[b], eta, a), L.ge_type4(t[b], A[b]))
        tol = method_tol(a, P)
        assert L.rel_err(S_gpu[b], L.ge_type5(t[b], s[b])) < e5 + tol
        assert L.rel_err(a_gpu[b], L.ge_type4(t[b], A[b])) < e4 + tol


def test_full_size_batch_sampled(env):
    """64 problems of P = 1024 at eta = 6 (the benchmarked shape), two checked
    against the oracle."""
    torch, NU, _ = env
    B, P, eta, mu = 64, 1024, 6, 1e-7
    a = NU.damping_for(mu, eta, P)
    t = inst(B, P, 2024)
    s = cn(np.random.default_rng(6), (B, P))
    S_gpu = NU.nufft_type5(dev(torch, t), dev(torch, s), eta, a).cpu().numpy()
    assert np.all(np.isfinite(S_gpu))
    for b in (0, B - 1):
        assert L.rel_err(S_gpu[b], L.type5_method(t[b], s[b], eta, a)) < method_tol(a, P)


def test_errors_are_reported_before_launch(env):
    torch, NU, nat = env
    lib = nat.load()
    t = dev(torch, inst(1, 64, 1))
    x = dev(torch, cn(np.random.default_rng(1), (1, 64)))
    y = torch.empty_like(x)
    ws = torch.empty(NU.nufft_workspace_size(1, 64, 6), dtype=torch.uint8, device="cuda")
    P = NU._ptr
    assert lib.nufft_type5(P(t), P(x), P(y), 1, 48, 6, 0.01, P(ws), ws.numel(), None) == nat.TF_EUNSUPPORTED
    assert lib.nufft_type5(P(t), P(x), P(y), 1, 64, 17, 0.01, P(ws), ws.numel(), None) == nat.TF_EUNSUPPORTED
    assert lib.nufft_type5(P(t), P(x), P(y), 1, 64, 6, 0.0, P(ws), ws.numel(), None) == nat.TF_EINVAL
    assert lib.nufft_type5(P(t), P(x), P(y), 1, 64, 6, 0.01, P(ws), 16, None) == nat.TF_EWORKSPACE
    assert lib.nudft_type1(P(t), P(x), P(y), 1, 0, 64, None) == nat.TF_EUNSUPPORTED
    assert lib.nudft_type2(P(t), P(x), P(y), 1, 65537, 64, None) == nat.TF_EUNSUPPORTED
    torch.cuda.synchronize()


@pytest.mark.parametrize("P,eta,mu", [(64, 2, 1e-4), (256, 1, 1e-4), (1024, 2, 1e-5)])
def test_refined_methods(env, P, eta, mu):
    """The refined methods of Sec. 5 against the oracle's refined methods, and
    their gain over one pass measured against Gaussian elimination."""
    torch, NU, _ = env
    B = 2
    a = NU.damping_for(mu, eta, P)
    t = inst(B, P, 5 * P + eta)
    rng = np.random.default_rng(3 * P + eta)
    s = cn(rng, (B, P))
    A = cn(rng, (B, P))
    S1 = NU.nufft_type5(dev(torch, t), dev(torch, s), eta, a, refine=True).cpu().numpy()
    a1 = NU.nufft_type4(dev(torch, t), dev(torch, A), eta, a, refine=True).cpu().numpy()
    tol = method_tol(a, P)
    for b in range(B):
        st = L.Setup(t[b], eta, a)
        assert L.rel_err(S1[b], L.type5_refined(t[b], s[b], eta, a, st)) < tol
        assert L.rel_err(a1[b], L.type4_refined(t[b], A[b], eta, a, st)) < tol
        e5 = L.rel_err(L.type5_method(t[b], s[b], eta, a, st), L.ge_type5(t[b], s[b]))
        e4 = L.rel_err(L.type4_method(t[b], A[b], eta, a, st), L.ge_type4(t[b], A[b]))
        assert L.rel_err(S1[b], L.ge_type5(t[b], s[b])) < 0.1 * e5 + tol
        assert L.rel_err(a1[b], L.ge_type4(t[b], A[b])) < 0.1 * e4 + tol


def test_refined_rejects_in_place(env):
    torch, NU, nat = env
    lib = nat.load()
    t = dev(torch, inst(1, 64, 1))
    x = dev(torch, cn(np.random.default_rng(1), (1, 64)))
    ws = torch.empty(NU.nufft_workspace_size(1, 64, 2), dtype=torch.uint8, device="cuda")
    P = NU._ptr
    assert lib.nufft_type4_refined(P(t), P(x), P(x), 1, 64, 2, 0.01, P(ws), ws.numel(), None) == nat.TF_EINVAL
    torch.cuda.synchronize()


# ------------------------------------------------------------ gridding NFFTs
@pytest.mark.parametrize("Q,R,unit", [(64, 64, False), (100, 1536, False), (1024, 6144, True), (1024, 2048, False)])
def test_gridding_type1(env, Q, R, unit):
    """Gridding type-1 against the gridding oracle and the exact sum; the Gaussian
    window is set for 1e-7 and the arithmetic is FP32."""
    from oracle import gridding as G
    torch, NU, _ = env
    B = 2
    t = inst(B, Q, 13 * Q + R)
    amp = None if unit else cn(np.random.default_rng(R), (B, Q))
    out = NU.nfft_type1(dev(torch, t), None if unit else dev(torch, amp), R).cpu().numpy()
    for b in range(B):
        a_b = np.ones(Q) if unit else amp[b]
        assert L.rel_err(out[b], G.type1(t[b], a_b, R)) < 2e-6
        assert L.rel_err(out[b], L.type1(t[b], a_b, R)) < 2e-6


@pytest.mark.parametrize("P,Q", [(64, 64), (1024, 1024), (2048, 300)])
def test_gridding_type2(env, P, Q):
    from oracle import gridding as G
    torch, NU, _ = env
    B = 2
    t = inst(B, Q, 17 * P + Q)
    c = cn(np.random.default_rng(P + 1), (B, P))
    out = NU.nfft_type2(dev(torch, t), dev(torch, c)).cpu().numpy()
    for b in range(B):
        assert L.rel_err(out[b], G.type2(c[b], t[b])) < 2e-6
        assert L.rel_err(out[b], L.type2(c[b], t[b])) < 2e-6


@pytest.mark.parametrize("P,eta,mu,refine", [(64, 6, 1e-7, False), (256, 4, 1e-7, False), (1024, 6, 1e-7, False),
                                             (256, 2, 1e-4, True)])
def test_methods_with_gridding(env, P, eta, mu, refine):
    """The type-5 / type-4 methods with every non-uniform sum by gridding, against
    the FP64 oracle of the methods (exact sums)."""
    torch, NU, _ = env
    B = 2
    a = NU.damping_for(mu, eta, P)
    t = inst(B, P, 23 * P + eta)
    rng = np.random.default_rng(P * eta)
    s = cn(rng, (B, P))
    A = cn(rng, (B, P))
    S = NU.nufft_type5(dev(torch, t), dev(torch, s), eta, a, gridding=True, refine=refine).cpu().numpy()
    x = NU.nufft_type4(dev(torch, t), dev(torch, A), eta, a, gridding=True, refine=refine).cpu().numpy()
    tol = 2e-5 * amp_of(a, P)
    f5 = L.type5_refined if refine else L.type5_method
    f4 = L.type4_refined if refine else L.type4_method
    for b in range(B):
        st = L.Setup(t[b], eta, a)
        assert L.rel_err(S[b], f5(t[b], s[b], eta, a, st)) < tol
        assert L.rel_err(x[b], f4(t[b], A[b], eta, a, st)) < tol


def test_gridding_shape_limits(env):
    torch, NU, nat = env
    # 2 eta P = 30720 is not a block-transform size
    assert NU.nufft_workspace_size(1, 1024, 15, NU.NUFFT_GRIDDING) == 0
    assert nat.load().nfft_workspace_size(1, 8) == 0
    assert nat.load().nfft_workspace_size(1, 1000) == 0      # 2000 = 16 x 125
    assert nat.load().nfft_workspace_size(1, 6144) > 0


@pytest.mark.parametrize("gridding", [False, True])
def test_setup_once_apply_many(env, gridding):
    """nufft_setup + nufft_apply (type 5, type 4, type 5 again, refined) reproduce
    the one-call solves bit for bit, and the applications leave the setup intact."""
    torch, NU, _ = env
    B, P, eta = 5, 256, 4
    a = NU.damping_for(1e-7, eta, P)
    t = dev(torch, inst(B, P, 41))
    rng = np.random.default_rng(42)
    s = dev(torch, cn(rng, (B, P)))
    A = dev(torch, cn(rng, (B, P)))
    print(f"case setup/apply gridding={gridding}", flush=True)
    ws = NU.nufft_setup(t, eta, a, gridding=gridding, refine=True)
    S5 = NU.nufft_apply(5, t, s, eta, a, ws, gridding=gridding).cpu().numpy()
    a4 = NU.nufft_apply(4, t, A, eta, a, ws, gridding=gridding).cpu().numpy()
    S5b = NU.nufft_apply(5, t, s, eta, a, ws, gridding=gridding).cpu().numpy()
    S5r = NU.nufft_apply(5, t, s, eta, a, ws, gridding=gridding, refine=True).cpu().numpy()
    a4r = NU.nufft_apply(4, t, A, eta, a, ws, gridding=gridding, refine=True).cpu().numpy()
    assert np.array_equal(S5, NU.nufft_type5(t, s, eta, a, gridding=gridding).cpu().numpy())
    assert np.array_equal(a4, NU.nufft_type4(t, A, eta, a, gridding=gridding).cpu().numpy())
    assert np.array_equal(S5b, S5)
    assert np.array_equal(S5r, NU.nufft_type5(t, s, eta, a, gridding=gridding, refine=True).cpu().numpy())
    assert np.array_equal(a4r, NU.nufft_type4(t, A, eta, a, gridding=gridding, refine=True).cpu().numpy())


@pytest.mark.parametrize("gridding", [False, True])
def test_graph_capture_of_solves(env, gridding):
    """After one eager run (twiddle tables are created on first use), a type-5 and a
    type-4 solve captured in a HIP graph replay bit-identically to the eager calls,
    with eager work between replays."""
    torch, NU, _ = env
    B, P, eta = 4, 256, 4
    a = NU.damping_for(1e-7, eta, P)
    t = dev(torch, inst(B, P, 51))
    rng = np.random.default_rng(52)
    s = dev(torch, cn(rng, (B, P)))
    A = dev(torch, cn(rng, (B, P)))
    S5 = torch.empty_like(s)
    a4 = torch.empty_like(A)
    ws = torch.empty(NU.nufft_workspace_size(B, P, eta, NU.NUFFT_GRIDDING if gridding else 0),
                     dtype=torch.uint8, device=s.device)

    def solves():
        NU.nufft_type5(t, s, eta, a, out=S5, workspace=ws, gridding=gridding)
        NU.nufft_type4(t, A, eta, a, out=a4, workspace=ws, gridding=gridding)

    solves()
    torch.cuda.synchronize()
    e5, e4 = S5.clone(), a4.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=torch.cuda.Stream()):
        solves()
    torch.cuda.synchronize()
    for rep in range(3):
        print(f"case nufft graph gridding={gridding} replay {rep}", flush=True)
        S5.zero_()
        a4.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(S5, e5) and torch.equal(a4, e4), rep
        NU.nudft_type1(t, s, 2 * P)            # eager work between replays
        torch.cuda.synchronize()


def test_empty_batch_is_a_no_op(env):
    torch, NU, nat = env
    lib = nat.load()
    assert lib.nufft_type5(None, None, None, 0, 64, 6, 0.01, None, 0, None) == nat.TF_OK
    assert lib.nudft_type1(None, None, None, 0, 64, 64, None) == nat.TF_OK
    assert lib.nudft_type2(None, None, None, 0, 64, 64, None) == nat.TF_OK
    assert lib.nfft_type1(None, None, None, 0, 64, 64, None, 0, None) == nat.TF_OK
    torch.cuda.synchronize()
