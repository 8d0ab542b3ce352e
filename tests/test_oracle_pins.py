"""The FP64 oracle against what the paper and the mathematics fix (CPU only)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import pins

# ----------------------------------------------------------------- oracle wrappers
fwd = O.forward
inv = O.inverse


def adj(ybar, taps, S):
    return O.adjoint(ybar, taps, S)


@pytest.mark.parametrize("pin", pins.ALL_FWD_PINS, ids=lambda p: p.__name__)
def test_forward_pins(pin):
    pin(fwd)


@pytest.mark.parametrize("pin", pins.ALL_PAIR_PINS, ids=lambda p: p.__name__)
def test_pair_pins(pin):
    pin(fwd, inv)


def test_adjoint_pin():
    pins.pin_adjoint(fwd, adj)


def test_gaussian_elimination_pin():
    pins.pin_gaussian_elimination(inv)


def test_explicit_matrix_and_transpose():
    """Brute-force matrix form on tiny blocks: forward = A S, adjoint = A^H ybar."""
    rng = np.random.default_rng(3)
    for N in (1, 2, 5, 12):
        taps = rng.uniform(0.5, 1.5, N)
        A = pins.explicit_matrix(taps)
        S = rng.normal(size=(2, N)) + 1j * rng.normal(size=(2, N))
        assert pins.rel_l2(fwd(S, taps), S @ A.T) < 1e-13
        Sbar, _ = O.adjoint(S, taps)
        assert pins.rel_l2(Sbar, S @ A.conj()) < 1e-13


# ----------------------------------------------------------------- extra oracle entry points
def test_inverse_counts_zero_taps():
    """The log-series filter of eq. (41) has a zero at n = 0, so its inverse is singular."""
    from paper_1604_06236_amd.workloads import log_series_taps
    N = 40
    taps = log_series_taps(N, 0.05)
    y = np.ones((3, N), complex)
    S, nz = O.inverse(y, taps, return_zero_count=True)
    assert nz == 3
    assert not np.all(np.isfinite(S[:, 0]))
    assert np.all(np.isfinite(S[:, 1:]))


def test_inverse_adjoint_is_transpose_and_tap_derivative():
    rng = np.random.default_rng(5)
    N = 24
    taps = rng.uniform(0.5, 1.5, N)
    y = rng.normal(size=(2, N)) + 1j * rng.normal(size=(2, N))
    g = rng.normal(size=(2, N)) + 1j * rng.normal(size=(2, N))
    Shat = O.inverse(y, taps)
    ybar, tb = O.inverse_adjoint(g, taps, Shat)
    # <g, inv(y)> = <inv^H g, y>
    assert abs(np.vdot(g, Shat) - np.vdot(ybar, y)) < 1e-12 * abs(np.vdot(g, Shat))
    h = 1e-6
    fd = np.empty(N)
    for n in range(N):
        tp = taps.copy(); tp[n] += h
        tm = taps.copy(); tm[n] -= h
        fd[n] = (np.vdot(g, O.inverse(y, tp)).real - np.vdot(g, O.inverse(y, tm)).real) / (2 * h)
    assert np.max(np.abs(tb - fd)) < 1e-6 * np.max(np.abs(fd))


def test_decimated_is_coset_zero_and_its_adjoint():
    rng = np.random.default_rng(6)
    for K, M in ((16, 5), (8, 15), (4, 1)):
        N = K * M
        taps = rng.uniform(0.5, 1.5, N)
        S = rng.normal(size=(3, N)) + 1j * rng.normal(size=(3, N))
        d = O.decimated(S, taps, K)
        # eq. (7) with numpy's IFFT
        folded = (taps * S).reshape(3, M, K).sum(axis=1)
        assert pins.rel_l2(d, K * np.fft.ifft(folded, axis=-1)) < 1e-13
        assert pins.rel_l2(d, O.forward(S, taps)[:, ::M]) < 1e-13
        yb = rng.normal(size=(3, K)) + 1j * rng.normal(size=(3, K))
        Sbar = O.decimated_adjoint(yb, taps, N)
        assert abs(np.vdot(yb, d) - np.vdot(Sbar, S)) < 1e-12 * abs(np.vdot(yb, d))


def test_log_series_decimated_gives_v_on_a_uniform_grid():
    """eq. (28): v(q/P) = sum_p log(1 - e^{j2pi(q/P - t_p + ja)}) is the nonuniform
    convolution of g (eq. (41), R = eta P) with the delta train of eq. (14).  For
    instants t_p on a uniform fine grid i/(eta P) the type-1 spectrum A(n) is the
    DFT of the train, and eq. (7) is the decimated transform."""
    from paper_1604_06236_amd.workloads import log_series_taps
    P, eta, a = 16, 6, 0.04
    R = eta * P
    idx = np.array([0, 5, 17, 40, 41, 77, 90])                    # occupied fine-grid points
    t = idx / R
    train = np.zeros(R, complex)
    train[idx] = 1.0
    A = np.fft.fft(train)                                          # A(n) = sum_p e^{-j2pi n t_p}
    v = O.decimated(A[None, :], log_series_taps(R, a), P)[0]
    q = np.arange(P)
    exact = np.array([np.sum(np.log(1 - np.exp(2j * np.pi * (qq / P - t)) * math.exp(-2 * math.pi * a)))
                      for qq in q])
    mu_bound = len(idx) * math.exp(-2 * math.pi * R * a) / (R * (1 - math.exp(-2 * math.pi * a)))
    assert np.max(np.abs(v - exact)) <= mu_bound + 1e-12


def test_ragged_matches_uniform():
    rng = np.random.default_rng(7)
    Ns = np.array([5, 12, 80, 7], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(Ns)[:-1]])
    tot = int(Ns.sum())
    S = rng.normal(size=tot) + 1j * rng.normal(size=tot)
    taps = rng.uniform(0.5, 1.5, tot)
    y = O.forward_ragged(Ns, off, off, S, taps)
    back = O.inverse_ragged(Ns, off, off, y, taps)
    Sbar, tb = O.adjoint_ragged(Ns, off, off, y, taps, S)
    for b, N in enumerate(Ns):
        sl = slice(off[b], off[b] + N)
        assert pins.rel_l2(y[sl], O.forward(S[None, sl], taps[sl])[0]) < 1e-14
        assert pins.rel_l2(back[sl], S[sl]) < 1e-13
        sb, t1 = O.adjoint(y[None, sl], taps[sl], S[None, sl])
        assert pins.rel_l2(Sbar[sl], sb[0]) < 1e-14
        assert pins.rel_l2(tb[sl], t1) < 1e-14


def test_conditioning_grows_with_damping():
    """The damping filter's inverse amplifies rounding by about e^{2 pi (N-1) a}
    (the attenuation trade-off of Sec. 5).  Perturb y at the 1e-12 level and
    watch the recovered coefficients."""
    rng = np.random.default_rng(8)
    N = 64
    S = rng.normal(size=(1, N)) + 1j * rng.normal(size=(1, N))
    errs = []
    for a in (0.0, 0.02, 0.05):
        taps = np.exp(-2 * math.pi * a * np.arange(N))
        y = O.forward(S, taps)
        noise = 1e-12 * np.linalg.norm(y) / math.sqrt(2 * N) * (
            rng.normal(size=y.shape) + 1j * rng.normal(size=y.shape))
        errs.append(pins.rel_l2(O.inverse(y + noise, taps), S))
        growth = math.exp(2 * math.pi * (N - 1) * a)
        assert errs[-1] < 50 * 1e-12 * growth
    assert errs[0] < errs[1] < errs[2]
    assert errs[2] / errs[0] > 0.01 * math.exp(2 * math.pi * (N - 1) * 0.05)


# ----------------------------------------------------------------- the pins catch mistakes
# Each mutant is a plausible bug planted in a copy of the oracle (on the CPU); at
# least one pin must reject it.
def _conj_sign(S, taps):                   # wrong exponent sign
    return O.forward(S.conj(), taps).conj()


def _taps_at_output(S, taps):              # filter applied to the wrong index
    return O.forward(S, np.ones_like(taps)) * taps


def _dropped_taps(S, taps):                # filter multiply dropped
    return O.forward(S, np.ones_like(taps))


def _normalised(S, taps):                  # spurious 1/N
    return O.forward(S, taps) / np.asarray(S).shape[-1]


def _index_reversed(S, taps):              # u -> -u (transposed/reversed operand)
    y = O.forward(S, taps)
    return np.roll(y[:, ::-1], 1, axis=1)


def _off_by_one_twiddle(S, taps):          # exponent (n+1) u instead of n u
    y = O.forward(S, taps)
    N = y.shape[-1]
    return y * np.exp(2j * np.pi * np.arange(N) / N)


MUTANTS = [_conj_sign, _taps_at_output, _dropped_taps, _normalised, _index_reversed,
           _off_by_one_twiddle]


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda f: f.__name__)
def test_pins_reject_mutant(mutant):
    caught = []
    for pin in pins.ALL_FWD_PINS:
        try:
            pin(mutant)
        except AssertionError:
            caught.append(pin.__name__)
    for pin in pins.ALL_PAIR_PINS:
        try:
            pin(mutant, inv)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin rejects {mutant.__name__}"


def _inv_wrong_scale(y, taps):
    return O.inverse(y, taps) * np.asarray(y).shape[-1]


def _inv_taps_mult(y, taps):
    return O.inverse(y, np.ones_like(taps)) * taps


def _adj_no_conj(ybar, taps, S):
    Sbar, tb = O.adjoint(np.conj(ybar), taps, S)
    return Sbar, tb


def _adj_tap_sign(ybar, taps, S):
    Sbar, tb = O.adjoint(ybar, taps, S)
    return Sbar, -tb


@pytest.mark.parametrize("mutant", [_inv_wrong_scale, _inv_taps_mult], ids=lambda f: f.__name__)
def test_inverse_pins_reject_mutant(mutant):
    caught = 0
    for pin in (pins.pin_library_fft, pins.pin_impulse_dc, pins.pin_round_trip):
        try:
            pin(fwd, mutant)
        except AssertionError:
            caught += 1
    try:
        pins.pin_gaussian_elimination(mutant)
    except AssertionError:
        caught += 1
    assert caught


@pytest.mark.parametrize("mutant", [_adj_no_conj, _adj_tap_sign], ids=lambda f: f.__name__)
def test_adjoint_pin_rejects_mutant(mutant):
    with pytest.raises(AssertionError):
        pins.pin_adjoint(fwd, mutant)


# ----------------------------------------------------------------- FFT form of the oracle
def test_fft_form_matches_the_plain_sums():
    """oracle/fftref.py (numpy FFT as its one library step) equals the O(N^2) oracle on
    uniform batches with shared and per-block taps, forward, inverse and adjoint."""
    from oracle import fftref as F
    from paper_1604_06236_amd import workloads as W
    rng = np.random.default_rng(21)
    for B, N in ((3, 80), (2, 1920), (4, 48), (1, 1)):
        S = W.cn01(rng, (B, N))
        y = W.cn01(rng, (B, N))
        for taps in (rng.uniform(0.5, 1.5, N), rng.uniform(0.5, 1.5, (B, N))):
            assert pins.rel_l2(F.forward(S, taps), O.forward(S, taps)) < 1e-12
            assert pins.rel_l2(F.inverse(y, taps), O.inverse(y, taps)) < 1e-12
            sb, tb = F.adjoint(y, taps, S)
            sb0, tb0 = O.adjoint(y, taps, S)
            assert pins.rel_l2(sb, sb0) < 1e-12
            assert np.linalg.norm(tb - tb0) <= 1e-12 * np.linalg.norm(tb0)


def test_fft_form_ragged_matches_the_plain_sums():
    from oracle import fftref as F
    from paper_1604_06236_amd import workloads as W
    lay, S, taps = W.make_ragged("ragged", nblocks=30)
    y = W.cn01(np.random.default_rng(5), lay.total)
    args = (lay.N, lay.x_off, lay.tap_off)
    assert pins.rel_l2(F.forward_ragged(*args, S, taps), O.forward_ragged(*args, S, taps)) < 1e-12
    assert pins.rel_l2(F.inverse_ragged(*args, y, taps), O.inverse_ragged(*args, y, taps)) < 1e-12
    sb, tb = F.adjoint_ragged(*args, y, taps, S)
    sb0, tb0 = O.adjoint_ragged(*args, y, taps, S)
    assert pins.rel_l2(sb, sb0) < 1e-12
    assert np.linalg.norm(tb - tb0) <= 1e-12 * np.linalg.norm(tb0)
    sb1, none = F.adjoint_ragged(*args, y, taps)
    assert none is None and pins.rel_l2(sb1, sb0) < 1e-12
