"""FP64 CPU oracle of the non-iterative type-5 and type-4 NFFT methods --
TEST INFRASTRUCTURE ONLY (tests, the package smoke check and the benchmark's
CPU baseline may use it; the product never does).

Plain numpy in float64 / complex128, one problem at a time, following the
steps of the type-5 flow (Sec. "Computation of the type-5 NFFT", the type-5
flow figure) and the type-4 flow (Sec. "Computation of the type-4 NFFT") in the
paper's order and notation.  The non-uniform transforms are exact O(P*R)
sums (no gridding), as the definitions eq. (32) and eq. (34) state them.

Notation: P instants t_p in [0, 1) (0-based arrays), damping a > 0,
oversampling eta (R = eta*P), z_p = exp(j 2 pi t_p).

Readings where the text is ambiguous:
* eq. (47) lists p = 1..P, but the method consumes {A(r)}_r^P, r = 0..P-1
  (eq. (37)); the type-4 system solved here uses p = 0..P-1, the exact
  Hermitian of the type-5 system eq. (48) (the duality of the numerical
  section).
* The IDFT is (1/P) sum e^{+j...}, so P*IDFT is the plain sum with the
  positive exponent (eq. (7), eq. (37)).
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- definitions
def type1(t, amp, R):
    """Type-1 NUDFT, eq. (32): A(r) = sum_q amp_q exp(-j 2 pi r t_q), r = 0..R-1."""
    t = np.asarray(t, np.float64)
    amp = np.asarray(amp, np.complex128)
    r = np.arange(R, dtype=np.float64)
    return np.exp(-2j * np.pi * np.outer(r, t)) @ amp


def type2(coef, t):
    """Type-2 NUDFT, eq. (34): s(t_q) = sum_p coef_p exp(+j 2 pi p t_q)."""
    t = np.asarray(t, np.float64)
    coef = np.asarray(coef, np.complex128)
    p = np.arange(coef.size, dtype=np.float64)
    return np.exp(2j * np.pi * np.outer(t, p)) @ coef


def type4_matrix(t):
    """Matrix of the type-4 system, eq. (47) with rows p = 0..P-1."""
    t = np.asarray(t, np.float64)
    return np.exp(-2j * np.pi * np.outer(np.arange(t.size), t))


def type5_matrix(t):
    """Matrix of the type-5 system, eq. (48): row q, column p -> exp(+j 2 pi p t_q)."""
    t = np.asarray(t, np.float64)
    return np.exp(2j * np.pi * np.outer(t, np.arange(t.size)))


def ge_type4(t, A):
    """Reference solution of eq. (47) by Gaussian elimination (LAPACK LU)."""
    return np.linalg.solve(type4_matrix(t), np.asarray(A, np.complex128))


def ge_type5(t, s):
    """Reference solution of eq. (48) by Gaussian elimination (LAPACK LU)."""
    return np.linalg.solve(type5_matrix(t), np.asarray(s, np.complex128))


def damping_for(mu, eta, P):
    """Damping a for a target truncation ratio mu, by inverting eq. (49):
    mu = exp(-2 pi (eta P - 1) a) / (eta P - 1)."""
    n = eta * P - 1
    return -np.log(mu * n) / (2 * np.pi * n)


def mu_of(a, eta, P):
    """Truncation ratio eq. (49)."""
    n = eta * P - 1
    return np.exp(-2 * np.pi * n * a) / n


# ---------------------------------------------------------------- method steps
def log_taps(R, a):
    """Coefficients of g(t), eq. (41): g_0 = 0, g_p = -(1/p) exp(-2 pi p a), 1 <= p < R
    (the series eq. (42) truncated at R)."""
    p = np.arange(R, dtype=np.float64)
    g = np.zeros(R)
    g[1:] = -np.exp(-2 * np.pi * p[1:] * a) / p[1:]
    return g


def v_samples(t, eta, a):
    """{v(q/P)}_q^P by eq. (28): the non-uniform convolution of g with the unit
    delta train z(t) (eq. (14)), evaluated as in eq. (26)-(7): a type-1 NUDFT of
    size R = eta P, the tap multiply, the fold onto P bins and P * IDFT."""
    P = len(t)
    R = eta * P
    Z = type1(t, np.ones(P), R)                 # spectrum of z(t) at 0..R-1
    B = log_taps(R, a) * Z
    fold = B.reshape(eta, P).sum(axis=0)        # sum over r of entry P r + p
    return P * np.fft.ifft(fold)


def kernel_samples(t, eta, a):
    """{L(exp(j 2 pi (q/P + j a)))}_q^P by eq. (29)."""
    t = np.asarray(t, np.float64)
    P = t.size
    return np.exp(1j * P * np.pi + 2j * np.pi * t.sum() + v_samples(t, eta, a))


def lagrange_coefficients(Lk, a):
    """{L_p}_p^{P+1} from the kernel samples, eq. (43) (DFT, removal of the alias of
    L_P = 1 at p = 0, compensation of the damping), with L_P = 1 appended."""
    Lk = np.asarray(Lk, np.complex128)
    P = Lk.size
    p = np.arange(P)
    D = np.fft.fft(Lk)
    D[0] -= P * np.exp(-2 * np.pi * P * a)
    L = D * np.exp(2 * np.pi * p * a) / P
    return np.concatenate([L, [1.0 + 0j]])


def derivative_samples(Lc, t):
    """{L'(exp(j 2 pi t_p))}_p^P: type-2 NUDFT of {(p+1) L_{p+1}}_p^P, eq. (16)."""
    Lc = np.asarray(Lc, np.complex128)
    P = Lc.size - 1
    return type2(np.arange(1, P + 1) * Lc[1:], t)


def h(x):
    """h(x) = 1 / (exp(j 2 pi x) - 1), eq. (17), for complex x."""
    return 1.0 / (np.exp(2j * np.pi * np.asarray(x)) - 1.0)


def h1(t, P, a):
    """h1(t) = sum_{p<P} exp(-2 pi p a) exp(j 2 pi p t), eq. (36) (series form)."""
    p = np.arange(P)
    return np.exp(-2 * np.pi * a * p) @ np.exp(2j * np.pi * np.outer(p, np.atleast_1d(t)))


def damping(P, a):
    """{exp(-2 pi p a)}_p^P, the invertible filter of eq. (8)."""
    return np.exp(-2 * np.pi * a * np.arange(P))


def weight_factor(t, Ld, a):
    """h(-P t_p + P j a) / (L'(exp(j 2 pi t_p)) exp(j 2 pi t_p)): the factor that
    turns samples s(t_p) into the delta-train weights of eq. (27) / eq. (40)."""
    t = np.asarray(t, np.float64)
    P = t.size
    return h(-P * t + 1j * P * a) / (np.asarray(Ld) * np.exp(2j * np.pi * t))


class Setup:
    """The part of both methods that depends on the instants only: kernel samples
    (eq. (28), eq. (29)), Lagrange coefficients (eq. (43)) and derivative samples
    (eq. (16))."""

    def __init__(self, t, eta, a):
        self.t = np.asarray(t, np.float64)
        self.P = self.t.size
        self.eta, self.a = int(eta), float(a)
        self.Lk = kernel_samples(self.t, self.eta, self.a)
        self.Lc = lagrange_coefficients(self.Lk, self.a)
        self.Ld = derivative_samples(self.Lc, self.t)
        self.wf = weight_factor(self.t, self.Ld, self.a)


def type5_method(t, s, eta, a, setup: Setup | None = None):
    """Coefficients {S_p} from samples {s(t_p)} (type-5 flow):
    weights eq. (27) -> type-1 NUDFT and eq. (37) filter/IDFT (the sum eq. (25))
    -> product with the kernel samples eq. (30) -> eq. (31)."""
    st = setup or Setup(t, eta, a)
    P, a = st.P, st.a
    w = np.asarray(s, np.complex128) * st.wf                       # eq. (27) a_p
    sigma = P * np.fft.ifft(damping(P, a) * type1(st.t, w, P))      # eq. (25) via eq. (37)
    s_shift = st.Lk * sigma                                         # eq. (30)
    return np.exp(2 * np.pi * a * np.arange(P)) * np.fft.fft(s_shift) / P   # eq. (31)


def type4_method(t, A, eta, a, setup: Setup | None = None):
    """Amplitudes {a_p} from spectral samples {A(r)}_r^P (type-4 flow):
    eq. (37) -> eq. (30) -> eq. (31) -> type-2 NUDFT -> eq. (40)."""
    st = setup or Setup(t, eta, a)
    P, a = st.P, st.a
    sigma = P * np.fft.ifft(damping(P, a) * np.asarray(A, np.complex128))   # eq. (37)
    s_shift = st.Lk * sigma                                                 # eq. (30)
    S = np.exp(2 * np.pi * a * np.arange(P)) * np.fft.fft(s_shift) / P      # eq. (31)
    return type2(S, st.t) * st.wf                                           # eq. (40)


def type4_refined(t, A, eta, a, setup: Setup | None = None):
    """Refined type-4 method (Sec. 5, eq. (44)-(46)): a first pass a0, the type-1
    sum of a0 minus the data (the error the method left in the spectrum, step 1-2),
    the method applied to that residual (step 3), subtracted from a0 (step 4)."""
    st = setup or Setup(t, eta, a)
    A = np.asarray(A, np.complex128)
    a0 = type4_method(t, A, eta, a, st)
    resid = type1(st.t, a0, st.P) - A
    return a0 - type4_method(t, resid, eta, a, st)


def type5_refined(t, s, eta, a, setup: Setup | None = None):
    """Refined type-5 method (the same residual correction, with the type-2
    evaluation of eq. (34) as the forward map)."""
    st = setup or Setup(t, eta, a)
    s = np.asarray(s, np.complex128)
    S0 = type5_method(t, s, eta, a, st)
    resid = type2(S0, st.t) - s
    return S0 - type5_method(t, resid, eta, a, st)


def rel_err(x, ref):
    """Relative quadratic-norm error of the numerical section."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
