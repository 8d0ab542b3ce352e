"""Gradients through the autograd Functions (adjoint kernels) against the FP64
oracle's transpose and finite differences.

PyTorch convention: for a real loss L and complex input z, z.grad = dL/dRe z +
j dL/dIm z.  For y = T_taps(S): S.grad = T^H y.grad (the oracle's adjoint) and
taps.grad_n = Re(conj(S_n) W_n), W = DFT(y.grad).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_06236_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def torch_T():
    import torch
    assert torch.cuda.is_available()
    from paper_1604_06236_amd import transform
    return torch, transform


def _leaf(torch, x, dtype=None):
    return torch.tensor(np.ascontiguousarray(x), device="cuda", dtype=dtype, requires_grad=True)


@pytest.mark.parametrize("K,M,shared", [(16, 5, True), (32, 3, False), (256, 9, True)])
def test_forward_gradients_match_oracle_transpose(torch_T, K, M, shared):
    torch, T = torch_T
    B, N = 5, K * M
    rng = np.random.default_rng(K)
    S = W.qam(rng, 16, (B, N)).astype(np.complex64)
    taps = (W.rc_taps(N, 0.3) if shared else np.stack([W.rc_taps(N, a) for a in (0.2, 0.4, 0.5, 0.7, 0.9)]))
    taps = taps.astype(np.float32)
    g = W.cn01(rng, (B, N)).astype(np.complex64)
    S_t, taps_t = _leaf(torch, S), _leaf(torch, taps)
    y = T.forward(S_t, taps_t, K, M)
    loss = (torch.conj(torch.from_numpy(g).cuda()) * y).real.sum()      # L = Re <g, y>
    loss.backward()
    Sbar_ref, tb_ref = O.adjoint(g, taps, S)
    assert rel(S_t.grad.cpu().numpy(), Sbar_ref) < 1e-5
    assert rel(taps_t.grad.cpu().numpy(), tb_ref) < 1e-5


@pytest.mark.parametrize("K,M,shared", [(16, 5, True), (64, 3, False)])
def test_inverse_gradients_match_oracle(torch_T, K, M, shared):
    torch, T = torch_T
    B, N = 4, K * M
    rng = np.random.default_rng(3 * K)
    y = W.cn01(rng, (B, N)).astype(np.complex64)
    taps = (W.rc_taps(N, 0.5) if shared else np.stack([W.rc_taps(N, a) for a in (0.2, 0.4, 0.6, 0.8)]))
    taps = taps.astype(np.float32)
    g = W.cn01(rng, (B, N)).astype(np.complex64)
    y_t, taps_t = _leaf(torch, y), _leaf(torch, taps)
    S = T.inverse(y_t, taps_t, K, M)
    loss = (torch.conj(torch.from_numpy(g).cuda()) * S).real.sum()
    loss.backward()
    Shat = O.inverse(y, taps)
    yb_ref, tb_ref = O.inverse_adjoint(g, taps, Shat)
    assert rel(y_t.grad.cpu().numpy(), yb_ref) < 1e-5
    assert rel(taps_t.grad.cpu().numpy(), tb_ref) < 1e-5
    # central finite differences of the FP64 oracle loss on a few taps
    t64 = taps.astype(np.float64)
    for n in (0, 7, N - 1):
        h = 1e-6
        tp, tm = t64.copy(), t64.copy()
        if shared:
            tp[n] += h
            tm[n] -= h
            fd = (np.vdot(g, O.inverse(y, tp)).real - np.vdot(g, O.inverse(y, tm)).real) / (2 * h)
            got = taps_t.grad.cpu().numpy()[n]
        else:
            tp[1, n] += h
            tm[1, n] -= h
            fd = (np.vdot(g, O.inverse(y, tp)).real - np.vdot(g, O.inverse(y, tm)).real) / (2 * h)
            got = taps_t.grad.cpu().numpy()[1, n]
        assert abs(got - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-4 * np.abs(tb_ref).max()


def test_differentiation_workload_loss(torch_T):
    """L(x, taps) = || inverse(forward(x) + noise) - x ||^2 on a slice of the
    differentiation workload (K=256, M=9, 16-QAM, RC roll-off 0.3, noise at
    20 dB below the unit signal power).  Since inverse(forward(x)) = x the loss
    equals || T^{-1} noise ||^2: its x-gradient vanishes and its tap gradient is
    -2 |W_n|^2 / (N^2 taps_n^3) summed over blocks, W = DFT(noise)."""
    torch, T = torch_T
    cfg = W.CONFIGS["differentiation"]
    K, M = cfg.K, cfg.M
    N = K * M
    x_h, taps_h = W.make_uniform(cfg, nblocks=64)
    B = x_h.shape[0]
    noise_h = W.awgn(np.random.default_rng(55), (B, N), 10 ** (-20 / 10)).astype(np.complex64)
    x_t, taps_t = _leaf(torch, x_h), _leaf(torch, taps_h)
    noise = torch.from_numpy(noise_h).cuda()
    y = T.forward(x_t, taps_t, K, M) + noise
    xr = T.inverse(y, taps_t, K, M)
    loss = ((xr - x_t).abs() ** 2).sum()
    loss.backward()
    # closed form from the oracle: T^{-1} noise = W / (N taps)
    u = O.inverse(noise_h, taps_h)                     # W_n / (N taps_n), per block
    t64 = taps_h.astype(np.float64)
    expect_taps = np.sum(-2.0 * np.abs(u) ** 2 / t64, axis=0)
    expect_loss = float(np.sum(np.abs(u) ** 2))
    assert abs(loss.item() - expect_loss) < 1e-4 * expect_loss
    assert rel(taps_t.grad.cpu().numpy(), expect_taps) < 1e-4
    # the x-gradient is zero analytically; numerically it is at rounding level
    gx = x_t.grad.cpu().numpy()
    scale = np.linalg.norm(2 * u.ravel())              # magnitude of each of the two cancelling terms
    assert np.linalg.norm(gx.ravel()) < 1e-5 * scale


def test_x_gradients_on_separate_losses(torch_T):
    """x-gradients of ||forward(x) - y0||^2 and ||inverse(y) - x0||^2 against the
    oracle: 2 T^H (T x - y0) and 2 T^{-H} (T^{-1} y - x0)."""
    torch, T = torch_T
    K, M, B = 256, 9, 6
    N = K * M
    rng = np.random.default_rng(8)
    x = W.qam(rng, 16, (B, N)).astype(np.complex64)
    y0 = W.cn01(rng, (B, N)).astype(np.complex64) * 10
    taps = W.rc_taps(N, 0.3).astype(np.float32)
    x_t = _leaf(torch, x)
    taps_t = torch.from_numpy(taps).cuda()
    loss = ((T.forward(x_t, taps_t, K, M) - torch.from_numpy(y0).cuda()).abs() ** 2).sum()
    loss.backward()
    r = O.forward(x, taps) - y0
    gref, _ = O.adjoint(2 * r, taps)
    assert rel(x_t.grad.cpu().numpy(), gref) < 1e-5
    y = O.forward(x, taps).astype(np.complex64)
    x0 = W.qam(rng, 16, (B, N)).astype(np.complex64)
    y_t = _leaf(torch, y)
    loss = ((T.inverse(y_t, taps_t, K, M) - torch.from_numpy(x0).cuda()).abs() ** 2).sum()
    loss.backward()
    r = O.inverse(y, taps) - x0
    gref, _ = O.inverse_adjoint(2 * r, taps)
    assert rel(y_t.grad.cpu().numpy(), gref) < 1e-5
