"""FFT form of the oracle's definitions, for full-size batches -- TEST
INFRASTRUCTURE ONLY (tests, the package smoke check and the benchmark's CPU
baseline may use it; the product never does).

The plain O(N^2) sums of oracle.c cannot cover batches of 10^4 blocks of up to
15360 points in seconds.  The same definitions with numpy's FFT (float64 /
complex128) as the one library step do:

  forward   y_u  = sum_n Lambda_n S_n e^{+j 2 pi n u/N}       = N * ifft(Lambda S)      (eq. (6) on u/N)
  inverse   S_n  = (N Lambda_n)^{-1} sum_u y_u e^{-j 2 pi n u/N} = fft(y) / (N Lambda)  (eq. (31))
  adjoint   W_n  = sum_u ybar_u e^{-j 2 pi n u/N} = fft(ybar);
            Sbar = Lambda W,  Lambdabar = Re(conj(S) W)

numpy's fft is the unnormalised negative-exponent DFT of eq. (0) and its ifft
carries 1/N, so no step here is more than the definition.  Pinned against the
O(N^2) oracle in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import numpy as np


def _blocks(x):
    return np.asarray(x, dtype=np.complex128)


def forward(S, taps):
    """[B, N] coefficients, taps [N] (shared) or [B, N] -> [B, N] samples."""
    S = _blocks(S)
    N = S.shape[-1]
    return N * np.fft.ifft(np.asarray(taps, np.float64) * S, axis=-1)


def inverse(y, taps):
    y = _blocks(y)
    N = y.shape[-1]
    with np.errstate(all="ignore"):
        return np.fft.fft(y, axis=-1) / (N * np.asarray(taps, np.float64))


def adjoint(ybar, taps, S=None):
    """(Sbar, tapbar); tapbar is summed over blocks when the taps are shared."""
    W = np.fft.fft(_blocks(ybar), axis=-1)
    taps = np.asarray(taps, np.float64)
    sbar = taps * W
    tb = None
    if S is not None:
        tb = np.real(np.conj(_blocks(S)) * W)
        if taps.ndim == 1:
            tb = tb.sum(axis=0)
    return sbar, tb


def _ragged(fn, N, x_off, tap_off, x, taps, *extra):
    """Apply a uniform function block by block over a flat ragged layout (blocks of one
    size are batched together)."""
    N = np.asarray(N, np.int64)
    x_off = np.asarray(x_off, np.int64)
    tap_off = np.asarray(tap_off, np.int64)
    x = np.asarray(x)
    taps = np.asarray(taps, np.float64)
    outs = None
    for n in np.unique(N):
        idx = np.nonzero(N == n)[0]
        xi = np.stack([x[o:o + n] for o in x_off[idx]])
        ti = np.stack([taps[o:o + n] for o in tap_off[idx]])
        ei = [np.stack([np.asarray(e)[o:o + n] for o in x_off[idx]]) for e in extra]
        res = fn(xi, ti, *ei)
        res = res if isinstance(res, tuple) else (res,)
        if outs is None:
            outs = [np.zeros(x.shape, dtype=np.complex128 if np.iscomplexobj(r) else np.float64)
                    for r in res]
        for k, r in enumerate(res):
            for row, o in zip(r, x_off[idx]):
                outs[k][o:o + n] = row
    return tuple(outs) if outs is not None else ()


def forward_ragged(N, x_off, tap_off, S, taps):
    return _ragged(forward, N, x_off, tap_off, S, taps)[0]


def inverse_ragged(N, x_off, tap_off, y, taps):
    return _ragged(inverse, N, x_off, tap_off, y, taps)[0]


def adjoint_ragged(N, x_off, tap_off, ybar, taps, S=None):
    """(Sbar, per-block tapbar laid out like the coefficients, or None)."""
    if S is None:
        return _ragged(lambda y, t: adjoint(y, t)[0], N, x_off, tap_off, ybar, taps)[0], None
    return _ragged(adjoint, N, x_off, tap_off, ybar, taps, S)
