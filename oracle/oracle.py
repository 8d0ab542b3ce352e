"""Python face of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package smoke check and the benchmark's CPU baseline may
import this module.  It builds `oracle.c` with gcc (no fast-math, OpenMP over
blocks) into `liboracle.so` next to it and wraps the entry points for numpy
arrays.  Inputs are upcast to complex128/float64 first, so the GPU path and
the oracle see the same values.

The definitions (per block of N points, omega = exp(+j 2 pi / N)) are those of
eq. (6) evaluated on the grid u/N, its inverse eq. (31) and their adjoints;
`oracle.c` states them in full.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile liboracle.so (gcc -O2 -fopenmp, IEEE arithmetic, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-ffp-contract=off", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        common = [ctypes.c_int64, _i64p, _i64p, _i64p]
        lib.oracle_forward.argtypes = common + [_f64p, _f64p, _f64p, ctypes.c_int]
        lib.oracle_inverse.argtypes = common + [_f64p, _f64p, _f64p, _i64p, ctypes.c_int]
        lib.oracle_adjoint.argtypes = common + [_f64p, _f64p, _f64p, _f64p, _f64p, ctypes.c_int]
        lib.oracle_inverse_adjoint.argtypes = common + [_f64p, _f64p, _f64p, _f64p, _f64p,
                                                        ctypes.c_int]
        dec = [ctypes.c_int64, _i64p, _i64p, _i64p, _i64p, _i64p]
        lib.oracle_decimated.argtypes = dec + [_f64p, _f64p, _f64p, ctypes.c_int]
        lib.oracle_decimated_adjoint.argtypes = dec + [_f64p, _f64p, _f64p, ctypes.c_int]
        for f in (lib.oracle_forward, lib.oracle_inverse, lib.oracle_adjoint,
                  lib.oracle_inverse_adjoint, lib.oracle_decimated, lib.oracle_decimated_adjoint,
                  lib.oracle_max_threads):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t=_f64p):
    return None if a is None else a.ctypes.data_as(t)


class _Layout:
    """Per-block sizes and offsets, uniform or ragged."""

    def __init__(self, N, x_off, tap_off, K=None):
        self.N = np.ascontiguousarray(N, dtype=np.int64)
        self.x_off = np.ascontiguousarray(x_off, dtype=np.int64)
        self.tap_off = np.ascontiguousarray(tap_off, dtype=np.int64)
        self.K = None if K is None else np.ascontiguousarray(K, dtype=np.int64)
        self.nblocks = int(self.N.size)
        self.total = int((self.x_off + self.N).max()) if self.nblocks else 0

    @classmethod
    def uniform(cls, B: int, N: int, shared: bool, K: Optional[int] = None):
        off = np.arange(B, dtype=np.int64) * N
        tap = np.zeros(B, dtype=np.int64) if shared else off.copy()
        return cls(np.full(B, N, dtype=np.int64), off, tap,
                   None if K is None else np.full(B, K, dtype=np.int64))


def _split_uniform(x, taps):
    x = _c128(x)
    if x.ndim != 2:
        raise ValueError("expected [B, N] blocks")
    B, N = x.shape
    taps = _f64(taps)
    shared = taps.ndim == 1
    if (shared and taps.shape != (N,)) or (not shared and taps.shape != (B, N)):
        raise ValueError("taps must be [N] (shared) or [B, N]")
    return x, taps, _Layout.uniform(B, N, shared)


def _nt(nthreads):
    return 0 if nthreads is None else int(nthreads)


# ------------------------------------------------------------------ uniform
def forward(S, taps, nthreads=None) -> np.ndarray:
    """y[b, u] = sum_n taps[n] S[b, n] exp(+j 2 pi n u / N)."""
    S, taps, lay = _split_uniform(S, taps)
    y = np.empty_like(S)
    _check(_load().oracle_forward(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                  _p(lay.tap_off, _i64p), _p(S.view(np.float64)), _p(taps),
                                  _p(y.view(np.float64)), _nt(nthreads)))
    return y


def inverse(y, taps, nthreads=None, return_zero_count=False):
    """S[b, n] = (N taps[n])^{-1} sum_u y[b, u] exp(-j 2 pi n u / N)."""
    y, taps, lay = _split_uniform(y, taps)
    S = np.empty_like(y)
    nz = np.zeros(1, dtype=np.int64)
    with np.errstate(all="ignore"):
        _check(_load().oracle_inverse(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                      _p(lay.tap_off, _i64p), _p(y.view(np.float64)), _p(taps),
                                      _p(S.view(np.float64)), _p(nz, _i64p), _nt(nthreads)))
    return (S, int(nz[0])) if return_zero_count else S


def adjoint(ybar, taps, S=None, nthreads=None, want_sbar=True):
    """(Sbar, tapbar) of the forward.  tapbar is summed over blocks when taps are shared."""
    ybar, taps, lay = _split_uniform(ybar, taps)
    Sbar = np.empty_like(ybar) if want_sbar else None
    tb = None
    if S is not None:
        S = _c128(S)
        if S.shape != ybar.shape:
            raise ValueError("S must match ybar")
        tb = np.empty(ybar.shape, dtype=np.float64)
    _check(_load().oracle_adjoint(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                  _p(lay.tap_off, _i64p), _p(ybar.view(np.float64)), _p(taps),
                                  None if S is None else _p(S.view(np.float64)),
                                  None if Sbar is None else _p(Sbar.view(np.float64)),
                                  _p(tb), _nt(nthreads)))
    if tb is not None and taps.ndim == 1:
        tb = tb.sum(axis=0)
    return Sbar, tb


def inverse_adjoint(gbar, taps, Shat=None, nthreads=None):
    """(ybar, tapbar) of the inverse, given the inverse's output Shat for the tap term."""
    gbar, taps, lay = _split_uniform(gbar, taps)
    ybar = np.empty_like(gbar)
    tb = None
    if Shat is not None:
        Shat = _c128(Shat)
        tb = np.empty(gbar.shape, dtype=np.float64)
    with np.errstate(all="ignore"):
        _check(_load().oracle_inverse_adjoint(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                              _p(lay.tap_off, _i64p), _p(gbar.view(np.float64)),
                                              _p(taps),
                                              None if Shat is None else _p(Shat.view(np.float64)),
                                              _p(ybar.view(np.float64)), _p(tb), _nt(nthreads)))
    if tb is not None and taps.ndim == 1:
        tb = tb.sum(axis=0)
    return ybar, tb


def decimated(S, taps, K: int, nthreads=None) -> np.ndarray:
    """eq. (7): out[b, q] = sum_n taps[n] S[b, n] exp(+j 2 pi n q / K), q < K."""
    S, taps, lay = _split_uniform(S, taps)
    B, N = S.shape
    if N % K:
        raise ValueError("K must divide N")
    Ks = np.full(B, K, dtype=np.int64)
    yoff = np.arange(B, dtype=np.int64) * K
    out = np.empty((B, K), dtype=np.complex128)
    _check(_load().oracle_decimated(B, _p(lay.N, _i64p), _p(Ks, _i64p), _p(lay.x_off, _i64p),
                                    _p(lay.tap_off, _i64p), _p(yoff, _i64p),
                                    _p(S.view(np.float64)), _p(taps), _p(out.view(np.float64)),
                                    _nt(nthreads)))
    return out


def decimated_adjoint(ybar, taps, N: int, nthreads=None) -> np.ndarray:
    """Sbar[b, n] = taps[n] sum_q ybar[b, q] exp(-j 2 pi n q / K)."""
    ybar = _c128(ybar)
    B, K = ybar.shape
    taps = _f64(taps)
    shared = taps.ndim == 1
    lay = _Layout.uniform(B, N, shared)
    Ks = np.full(B, K, dtype=np.int64)
    yoff = np.arange(B, dtype=np.int64) * K
    Sbar = np.empty((B, N), dtype=np.complex128)
    _check(_load().oracle_decimated_adjoint(B, _p(lay.N, _i64p), _p(Ks, _i64p),
                                            _p(lay.x_off, _i64p), _p(lay.tap_off, _i64p),
                                            _p(yoff, _i64p), _p(ybar.view(np.float64)), _p(taps),
                                            _p(Sbar.view(np.float64)), _nt(nthreads)))
    return Sbar


# ------------------------------------------------------------------ ragged
def _ragged_layout(N, x_off, tap_off):
    return _Layout(N, x_off, tap_off)


def forward_ragged(N, x_off, tap_off, S, taps, nthreads=None) -> np.ndarray:
    """Ragged forward over a flat coefficient array; block b has N[b] points."""
    lay = _ragged_layout(N, x_off, tap_off)
    S = _c128(S)
    taps = _f64(taps)
    y = np.zeros_like(S)
    _check(_load().oracle_forward(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                  _p(lay.tap_off, _i64p), _p(S.view(np.float64)), _p(taps),
                                  _p(y.view(np.float64)), _nt(nthreads)))
    return y


def inverse_ragged(N, x_off, tap_off, y, taps, nthreads=None) -> np.ndarray:
    lay = _ragged_layout(N, x_off, tap_off)
    y = _c128(y)
    taps = _f64(taps)
    S = np.zeros_like(y)
    nz = np.zeros(1, dtype=np.int64)
    with np.errstate(all="ignore"):
        _check(_load().oracle_inverse(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                      _p(lay.tap_off, _i64p), _p(y.view(np.float64)), _p(taps),
                                      _p(S.view(np.float64)), _p(nz, _i64p), _nt(nthreads)))
    return S


def adjoint_ragged(N, x_off, tap_off, ybar, taps, S=None, nthreads=None):
    """(Sbar, per-block tapbar laid out like the coefficients)."""
    lay = _ragged_layout(N, x_off, tap_off)
    ybar = _c128(ybar)
    taps = _f64(taps)
    Sbar = np.zeros_like(ybar)
    tb = None
    if S is not None:
        S = _c128(S)
        tb = np.zeros(ybar.shape, dtype=np.float64)
    _check(_load().oracle_adjoint(lay.nblocks, _p(lay.N, _i64p), _p(lay.x_off, _i64p),
                                  _p(lay.tap_off, _i64p), _p(ybar.view(np.float64)), _p(taps),
                                  None if S is None else _p(S.view(np.float64)),
                                  _p(Sbar.view(np.float64)), _p(tb), _nt(nthreads)))
    return Sbar, tb


def _check(rc: int):
    if rc != 0:
        raise MemoryError("oracle: allocation failed")
