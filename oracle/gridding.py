"""FP64 CPU oracle of gridding type-1 / type-2 NFFTs -- TEST INFRASTRUCTURE ONLY
(tests, the package smoke check and the benchmark's CPU baseline may use it;
the product never does).

The paper describes the type-1 NFFT as one gridding operation plus one FFT at
oversampling factor two, and the type-2 NFFT as a weighting, an inverse FFT and
a short interpolation sum (Sec. 2, around eq. (32)-(34)), without naming the
window.  This oracle uses the Gaussian window of Dutt-Rokhlin /
Greengard-Lee ("Accelerating the nonuniform fast Fourier transform", 2004),
whose Fourier transform has a closed form, in plain numpy, one problem at a
time:

  fine grid n = 2 * (number of frequencies), g_tau(x) = exp(-x^2 / (4 tau))
  periodised, tau = ln(1/eps) / (2 pi^2 n^2) (the alias at k - n of the band
  edge k = n/4 is then eps times smaller), truncated to grid offsets
  -h+1 .. h around floor(n t) with h = ceil(sqrt(2) ln(1/eps) / pi) (the
  window has fallen to eps at h/n), and
  g_hat(k) = sqrt(4 pi tau) exp(-4 pi^2 k^2 tau).

The frequencies 0..R-1 of eq. (32) are handled as the centred band
-R/2..R/2-1 after modulating the amplitudes by exp(-j 2 pi (R/2) t).
"""
from __future__ import annotations

import math

import numpy as np


def params(R, eps=1e-7):
    """(n, tau, half): fine-grid size, Gaussian width, spreading half width (the
    window covers grid offsets -half+1 .. half around floor(n t))."""
    n = 2 * int(R)
    L = math.log(1.0 / eps)
    tau = L / (2 * math.pi ** 2 * n * n)
    half = int(math.ceil(math.sqrt(2.0) * L / math.pi))
    return n, tau, half


def g_hat(k, tau):
    return math.sqrt(4 * math.pi * tau) * np.exp(-4 * math.pi ** 2 * np.asarray(k, np.float64) ** 2 * tau)


def _window_rows(t, n, tau, half):
    """For every instant: the grid indices it touches and the window values there."""
    t = np.mod(np.asarray(t, np.float64), 1.0)
    x = n * t
    m0 = np.floor(x)
    j = np.arange(-half + 1, half + 1)
    m = (m0[:, None] + j[None, :]).astype(np.int64)
    d = (x[:, None] - m) / n                     # distance in units of the period
    w = np.exp(-d * d / (4 * tau))
    return np.mod(m, n), w


def type1(t, amp, R, eps=1e-7):
    """A(r) = sum_q amp_q exp(-j 2 pi r t_q), r < R, by gridding (spread, FFT,
    deconvolve)."""
    t = np.asarray(t, np.float64)
    amp = np.asarray(amp, np.complex128)
    n, tau, half = params(R, eps)
    c = amp * np.exp(-2j * math.pi * (R // 2) * t)          # centre the band
    idx, w = _window_rows(t, n, tau, half)
    grid = np.zeros(n, np.complex128)
    np.add.at(grid, idx.ravel(), (c[:, None] * w).ravel())
    F = np.fft.fft(grid) / n                                # trapezoid rule of the integral
    k = np.arange(R) - R // 2                               # centred frequency of output r
    return F[np.mod(k, n)] / g_hat(k, tau)


def type2(coef, t, eps=1e-7):
    """s(t_q) = sum_p coef_p exp(+j 2 pi p t_q) by gridding (deconvolve, inverse
    FFT, interpolate)."""
    t = np.asarray(t, np.float64)
    coef = np.asarray(coef, np.complex128)
    P = coef.size
    n, tau, half = params(P, eps)
    k = np.arange(P) - P // 2
    H = np.zeros(n, np.complex128)
    H[np.mod(k, n)] = coef / g_hat(k, tau)
    h = n * np.fft.ifft(H)                                  # h(m/n) = sum_k H_k e^{+j 2 pi k m / n}
    idx, w = _window_rows(t, n, tau, half)
    f = (h[idx] * w).sum(axis=1) / n                        # (1/n) sum_m g(t - m/n) h(m/n)
    return f * np.exp(2j * math.pi * (P // 2) * np.mod(t, 1.0))
