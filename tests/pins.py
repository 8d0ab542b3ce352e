"""Checks that pin a block-transform implementation to what the paper and the
mathematics fix, independently of how the implementation computes.

Each check takes callables `fwd(S, taps)`, `inv(y, taps)` (and, where needed,
`adj(ybar, taps, S) -> (Sbar, tapbar)`) operating on [B, N] complex arrays and
[N] real taps, and raises AssertionError when the pin is violated.  The same
checks are run against the real oracle (must pass) and against deliberately
broken copies of it (each must trip at least one check), see
test_oracle_pins.py.

Pins and the passages they come from:
  * library routine: with all taps 1 the forward is N * IFFT and the inverse is
    FFT / N (DFT of eq. (0); the IDFT's 1/P is fixed by eq. (7) and eq. (37));
  * the fold of eq. (7): coset u = M q equals K * IDFT_K of the folded,
    filtered spectrum, computed with numpy's FFT;
  * the four-step staging (filter, length-M DFT, coset twiddle, length-K DFT)
    written with numpy's FFT, for every coset;
  * impulse and DC responses of eq. (6);
  * Parseval, from eq. (0) and the IDFT normalisation;
  * the damping filter of eq. (8): its response to S = 1 is the closed form of
    h1 in eq. (36);
  * the truncated log series of eq. (41) reproduces log(1 - e^{j2pi(t+ja)}) of
    eq. (42) within the tail bound behind eq. (49);
  * the truncated series of eq. (20) reproduces h(t + ja) of eq. (17);
  * eq. (37): with M = 1 and damping taps, the transform of the type-1 spectrum
    A(r) of eq. (32) equals sum_p a_p h1(q/P - t_p);
  * the adjoint identity <T S, y> = <S, T^H y> (the Hermitian pairing of the
    type-4/type-5 duality, Sec. 6) and finite differences for the tap term;
  * Gaussian elimination (the paper's GE method, Sec. 6) on the forward's
    matrix reproduces the inverse.
"""
from __future__ import annotations

import math

import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return float(d / n) if n > 0 else float(d)


def _rand_blocks(rng, B, N):
    return rng.normal(size=(B, N)) + 1j * rng.normal(size=(B, N))


def _rand_taps(rng, N):
    # bounded away from zero so the inverse is well conditioned
    return rng.uniform(0.5, 1.5, size=N)


def _fwd1(fwd, S, taps):
    """Single-block helper: fwd on S[N] -> y[N]."""
    return np.asarray(fwd(np.asarray(S)[None, :], taps))[0]


# ---------------------------------------------------------------- pins
def pin_library_fft(fwd, inv, Ns=(1, 2, 3, 7, 16, 45, 80), tol=1e-12):
    rng = np.random.default_rng(11)
    for N in Ns:
        S = _rand_blocks(rng, 3, N)
        ones = np.ones(N)
        y = fwd(S, ones)
        assert rel_l2(y, N * np.fft.ifft(S, axis=-1)) < tol, f"forward != N*ifft at N={N}"
        back = inv(y, ones)
        assert rel_l2(back, np.fft.fft(y, axis=-1) / N) < tol, f"inverse != fft/N at N={N}"


def pin_fold_eq7(fwd, shapes=((16, 5), (8, 3), (4, 15), (1, 7), (32, 1)), tol=1e-12):
    """Coset m = 0 of the grid: y[M q] = K * IDFT_K{ sum_r taps[p+Kr] S[p+Kr] }."""
    rng = np.random.default_rng(12)
    for K, M in shapes:
        N = K * M
        S = _rand_blocks(rng, 2, N)
        taps = _rand_taps(rng, N)
        y = fwd(S, taps)
        folded = (taps * S).reshape(2, M, K).sum(axis=1)           # sum over r of index p + K r
        expect = K * np.fft.ifft(folded, axis=-1)
        assert rel_l2(y[:, ::M], expect) < tol, f"eq.(7) fold violated at K={K} M={M}"


def staged_numpy(S, taps, K, M):
    """The four-step form with numpy FFTs: filter, length-M DFT over r, coset
    twiddle exp(+j 2 pi p m / N), length-K DFT over p; output index u = M q + m."""
    S = np.asarray(S)
    B, N = S.shape
    Z = (taps * S).reshape(B, M, K)                     # Z[b, r, p] = Z_{p + K r}
    U = M * np.fft.ifft(Z, axis=1)                      # U[b, m, p] = sum_r Z e^{+j2pi rm/M}
    p = np.arange(K)[None, :]
    m = np.arange(M)[:, None]
    U = U * np.exp(2j * np.pi * ((p * m) % N) / N)[None]
    Y = K * np.fft.ifft(U, axis=2)                      # Y[b, m, q]
    return Y.transpose(0, 2, 1).reshape(B, N)           # u = M q + m


def pin_staged(fwd, shapes=((1, 1), (2, 3), (4, 5), (8, 7), (16, 9), (16, 15), (4, 16), (64, 3)),
               tol=1e-12):
    rng = np.random.default_rng(13)
    for K, M in shapes:
        N = K * M
        S = _rand_blocks(rng, 2, N)
        taps = _rand_taps(rng, N)
        assert rel_l2(fwd(S, taps), staged_numpy(S, taps, K, M)) < tol, \
            f"staged form differs at K={K} M={M}"


def pin_impulse_dc(fwd, inv, Ns=(5, 12, 80), tol=1e-12):
    rng = np.random.default_rng(14)
    for N in Ns:
        taps = _rand_taps(rng, N)
        u = np.arange(N)
        for n0 in sorted({0, 1, N // 2, N - 1}):
            S = np.zeros(N, complex)
            S[n0] = 1.0
            y = _fwd1(fwd, S, taps)
            expect = taps[n0] * np.exp(2j * np.pi * ((n0 * u) % N) / N)
            assert np.max(np.abs(y - expect)) < tol, f"impulse response wrong at N={N}, n0={n0}"
        c = 0.7 - 0.3j
        back = np.asarray(inv(np.full((1, N), c), taps))[0]
        expect = np.zeros(N, complex)
        expect[0] = c / taps[0]
        assert np.max(np.abs(back - expect)) < tol * abs(c / taps[0]), "DC inverse wrong"


def pin_parseval(fwd, Ns=(7, 80, 240), tol=1e-12):
    rng = np.random.default_rng(15)
    for N in Ns:
        S = _rand_blocks(rng, 4, N)
        taps = _rand_taps(rng, N)
        y = fwd(S, taps)
        lhs = np.sum(np.abs(y) ** 2, axis=-1)
        rhs = N * np.sum(np.abs(taps * S) ** 2, axis=-1)
        assert np.max(np.abs(lhs / rhs - 1)) < tol, f"Parseval violated at N={N}"


def pin_round_trip(fwd, inv, Ns=(3, 80, 128), tol=1e-12):
    rng = np.random.default_rng(16)
    for N in Ns:
        S = _rand_blocks(rng, 3, N)
        taps = _rand_taps(rng, N)
        assert rel_l2(inv(fwd(S, taps), taps), S) < tol, f"inverse(forward) != I at N={N}"
        assert rel_l2(fwd(inv(S, taps), taps), S) < tol, f"forward(inverse) != I at N={N}"


def damping_closed_form(N, a):
    """h1 of eq. (36) with P -> N, sampled at t = u/N (S = 1, taps exp(-2 pi n a))."""
    u = np.arange(N)
    e = np.exp(2j * np.pi * u / N) * math.exp(-2 * math.pi * a)
    return (1 - math.exp(-2 * math.pi * N * a)) / (1 - e)


def pin_damping_eq36(fwd, cases=((64, 0.01), (80, 0.002), (15, 0.05)), tol=1e-12):
    for N, a in cases:
        taps = np.exp(-2 * math.pi * a * np.arange(N))
        y = _fwd1(fwd, np.ones(N, complex), taps)
        assert rel_l2(y, damping_closed_form(N, a)) < tol, f"eq.(36) closed form at N={N}, a={a}"


def pin_log_series_eq42(fwd, cases=((64, 0.05), (128, 0.02), (240, 0.01))):
    """sum_{n=1}^{N-1} -e^{-2 pi n a}/n e^{j 2 pi n u/N} vs log(1 - e^{j 2 pi (u/N + ja)}).

    The dropped tail is bounded by sum_{n>=N} e^{-2 pi n a}/n <= e^{-2 pi N a}/(N(1-e^{-2 pi a})).
    """
    for N, a in cases:
        n = np.arange(N, dtype=float)
        taps = np.zeros(N)
        taps[1:] = -np.exp(-2 * math.pi * a * n[1:]) / n[1:]
        y = _fwd1(fwd, np.ones(N, complex), taps)
        z = np.exp(2j * np.pi * (np.arange(N) / N)) * math.exp(-2 * math.pi * a)
        exact = np.log(1 - z)
        bound = math.exp(-2 * math.pi * N * a) / (N * (1 - math.exp(-2 * math.pi * a)))
        err = np.max(np.abs(y - exact))
        assert err <= bound * (1 + 1e-6) + 1e-13, f"eq.(42) tail bound violated at N={N}, a={a}: {err} > {bound}"


def pin_h_series_eq20(fwd, cases=((64, 0.05), (100, 0.03))):
    for N, a in cases:
        taps = -np.exp(-2 * math.pi * a * np.arange(N))
        y = _fwd1(fwd, np.ones(N, complex), taps)
        z = np.exp(2j * np.pi * (np.arange(N) / N)) * math.exp(-2 * math.pi * a)
        exact = 1.0 / (z - 1.0)
        bound = math.exp(-2 * math.pi * N * a) / (1 - math.exp(-2 * math.pi * a))
        err = np.max(np.abs(y - exact))
        assert err <= bound * (1 + 1e-6) + 1e-13, f"eq.(20) bound violated at N={N}, a={a}"


def h1_closed(t, P, a):
    """h1(t) of eq. (36) in its closed form (e^{j2pi P(t+ja)} - 1)/(e^{j2pi(t+ja)} - 1)."""
    zt = np.exp(2j * np.pi * t) * math.exp(-2 * math.pi * a)
    zP = np.exp(2j * np.pi * P * t) * math.exp(-2 * math.pi * P * a)
    return (zP - 1) / (zt - 1)


def pin_eq37(fwd, cases=((16, 0.02), (64, 0.005))):
    """eq. (37): P * IDFT(e^{-2 pi r a} (.) A(r)) = {sum_p a_p h1(q/P - t_p)}_q, with
    A(r) = sum_p a_p e^{-j 2 pi r t_p} the type-1 spectrum of eq. (32)."""
    rng = np.random.default_rng(17)
    for P, a in cases:
        t = (np.arange(P) + rng.uniform(0, 0.6, P)) / P          # jittered grid, Sec. 6
        amp = (rng.normal(size=P) + 1j * rng.normal(size=P)) / math.sqrt(2)
        r = np.arange(P)
        A = np.exp(-2j * np.pi * np.outer(r, t)) @ amp           # brute-force NUDFT, eq. (32)
        taps = np.exp(-2 * math.pi * a * r)
        y = _fwd1(fwd, A, taps)
        q = np.arange(P)
        expect = np.array([np.sum(amp * h1_closed(qq / P - t, P, a)) for qq in q])
        assert rel_l2(y, expect) < 1e-11, f"eq.(37) violated at P={P}, a={a}"


def pin_adjoint(fwd, adj, Ns=(6, 45, 80), tol=1e-12):
    """<T S, y> = <S, T^H y> for the coefficient adjoint, and the tap term of
    the adjoint equals the derivative of Re<ybar, T_taps S> w.r.t. each tap."""
    rng = np.random.default_rng(18)
    for N in Ns:
        S = _rand_blocks(rng, 2, N)
        Y = _rand_blocks(rng, 2, N)
        taps = _rand_taps(rng, N)
        lhs = np.vdot(Y, fwd(S, taps))
        Sbar, tb = adj(Y, taps, S)
        rhs = np.vdot(Sbar, S)
        assert abs(lhs - rhs) < tol * abs(lhs) + 1e-300, f"adjoint identity fails at N={N}"
        # real-valued loss L(taps) = Re <Y, fwd(S, taps)> is linear in the taps, so a
        # central difference is exact up to rounding
        h = 1e-3
        fd = np.empty(N)
        for n in range(N):
            tp = taps.copy(); tp[n] += h
            tm = taps.copy(); tm[n] -= h
            fd[n] = (np.vdot(Y, fwd(S, tp)).real - np.vdot(Y, fwd(S, tm)).real) / (2 * h)
        assert np.max(np.abs(tb - fd)) < 1e-8 * np.max(np.abs(fd)), f"tap gradient fails at N={N}"


def explicit_matrix(taps):
    """A = F diag(taps), F[u, n] = exp(+j 2 pi (n u mod N)/N), for tiny N."""
    N = len(taps)
    u = np.arange(N)
    F = np.exp(2j * np.pi * (np.outer(u, u) % N) / N)
    return F * np.asarray(taps)[None, :]


def pin_gaussian_elimination(inv, Ns=(3, 8, 30), tol=1e-11):
    rng = np.random.default_rng(19)
    for N in Ns:
        taps = _rand_taps(rng, N)
        y = _rand_blocks(rng, 1, N)
        ge = np.linalg.solve(explicit_matrix(taps), y[0])
        assert rel_l2(np.asarray(inv(y, taps))[0], ge) < tol, f"inverse != GE at N={N}"


ALL_FWD_PINS = (pin_fold_eq7, pin_staged, pin_parseval, pin_damping_eq36,
                pin_log_series_eq42, pin_h_series_eq20, pin_eq37)
ALL_PAIR_PINS = (pin_library_fft, pin_impulse_dc, pin_round_trip)
