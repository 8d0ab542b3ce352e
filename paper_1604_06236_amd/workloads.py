"""Seeded synthetic inputs for the block transform.

This module only draws numbers: symbols, filter taps and block layouts. It
holds none of the transform's arithmetic, so both the GPU path and the CPU
oracle can be fed from it without sharing any of the method.

The transform evaluates a filtered trigonometric polynomial on a uniform grid
(the convolution of eq. (26) evaluated through eq. (6)/(7), and its invertible
form eq. (8)/(31)).  A block is N = K*M complex coefficients S_n together with N
real taps Lambda_n.  The paper fixes no data set; its own experiments draw
complex Gaussian amplitudes and jittered instants (Sec. 6, "Monte Carlo
trials").  The workloads below use the shapes named for the five standard
configurations and the following recipe:

* symbols: square M-QAM on the odd-integer grid, scaled to unit mean energy,
  indices uniform; or CN(0,1) (real and imaginary parts each N(0, 1/2));
* taps: raised-cosine (RC) or root-raised-cosine (RRC) spectra over the N
  frequency bins, nu_n = min(n, N-n)/N, normalised to unit energy in FP64 and
  rounded to FP32.  Their smallest value is 1/2 (RC) or 1/sqrt(2) (RRC) of the
  largest, so the filter is always invertible;
* the paper's own filters (damping exp(-2 pi n a) of eq. (8)/(36), the
  truncated log series of eq. (41), and the h-kernel series of eq. (20)) for
  the closed-form checks;
* seeds: numpy PCG64, one independent stream per purpose via SeedSequence.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Config", "CONFIGS", "rng_streams", "qam", "cn01", "rc_taps", "rrc_taps",
    "damping_taps", "log_series_taps", "h_series_taps", "RaggedLayout",
    "ragged_layout", "make_uniform", "make_ragged", "awgn",
    "jittered_instants",
]


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------
def rng_streams(seed: int, n: int) -> list:
    """`n` independent numpy Generators derived from one integer seed."""
    ss = np.random.SeedSequence(int(seed))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def qam(rng: np.random.Generator, order: int, size) -> np.ndarray:
    """Square `order`-QAM symbols (4, 16, 64, ...) with unit mean energy.

    Levels are the odd integers -(L-1), ..., -1, 1, ..., L-1 with L = sqrt(order);
    the mean energy of that grid is 2(L^2-1)/3, which is divided out.
    """
    L = int(round(math.sqrt(order)))
    if L * L != order or L < 2:
        raise ValueError(f"QAM order must be a perfect square >= 4, got {order}")
    levels = np.arange(-(L - 1), L, 2, dtype=np.float64)
    idx_re = rng.integers(0, L, size=size)
    idx_im = rng.integers(0, L, size=size)
    scale = 1.0 / math.sqrt(2.0 * (L * L - 1) / 3.0)
    return (levels[idx_re] + 1j * levels[idx_im]) * scale


def cn01(rng: np.random.Generator, size) -> np.ndarray:
    """Circular complex Gaussian CN(0, 1)."""
    s = math.sqrt(0.5)
    return rng.normal(0.0, s, size=size) + 1j * rng.normal(0.0, s, size=size)


def awgn(rng: np.random.Generator, size, sigma2: float) -> np.ndarray:
    """Complex white Gaussian noise CN(0, sigma2)."""
    return cn01(rng, size) * math.sqrt(sigma2)


# --------------------------------------------------------------------------
# filter taps
# --------------------------------------------------------------------------
def _freq_axis(N: int) -> np.ndarray:
    n = np.arange(N, dtype=np.float64)
    return np.minimum(n, N - n) / N           # in [0, 1/2]


def rc_taps(N: int, alpha: float, unit_energy: bool = True) -> np.ndarray:
    """Raised-cosine spectrum over the N bins (FP64).

    RC(nu) = 1 for nu <= (1-alpha)/2, else (1 + cos(pi (nu - (1-alpha)/2)/alpha))/2,
    with nu = min(n, N-n)/N <= 1/2, so RC >= 1/2 everywhere.
    """
    if not (0.0 < alpha <= 1.0):
        raise ValueError("roll-off must be in (0, 1]")
    nu = _freq_axis(N)
    edge = 0.5 * (1.0 - alpha)
    t = np.ones(N)
    hi = nu > edge
    t[hi] = 0.5 * (1.0 + np.cos(math.pi * (nu[hi] - edge) / alpha))
    if unit_energy:
        t = t / math.sqrt(float(np.sum(t * t)))
    return t


def rrc_taps(N: int, alpha: float, unit_energy: bool = True) -> np.ndarray:
    """Root-raised-cosine spectrum (square root of `rc_taps`), FP64."""
    t = np.sqrt(rc_taps(N, alpha, unit_energy=False))
    if unit_energy:
        t = t / math.sqrt(float(np.sum(t * t)))
    return t


def damping_taps(N: int, a: float) -> np.ndarray:
    """exp(-2 pi n a), the invertible damping filter of eq. (8) (and h1, eq. (36))."""
    return np.exp(-2.0 * math.pi * a * np.arange(N, dtype=np.float64))


def log_series_taps(N: int, a: float) -> np.ndarray:
    """Coefficients of g(t) in eq. (41): -exp(-2 pi n a)/n for 1 <= n < N, 0 at n = 0."""
    n = np.arange(N, dtype=np.float64)
    t = np.zeros(N)
    t[1:] = -np.exp(-2.0 * math.pi * a * n[1:]) / n[1:]
    return t


def h_series_taps(N: int, a: float) -> np.ndarray:
    """Truncated Fourier series of h(t + ja), eq. (20): -exp(-2 pi n a)."""
    return -damping_taps(N, a)


def jittered_instants(rng: np.random.Generator, P: int, jitter: float = 0.6) -> np.ndarray:
    """Instants p/P + U[0, jitter/P], the Monte Carlo grid of Sec. 6."""
    return (np.arange(P) + rng.uniform(0.0, jitter, size=P)) / P


# --------------------------------------------------------------------------
# standard configurations
# --------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    seed: int
    nblocks: int
    K: Optional[int]            # None for ragged
    M: Optional[int]
    symbols: str                # "qam4", "qam16", "qam64", "cn01"
    taps: str                   # "rc", "rrc"
    alpha: Optional[float]      # None: drawn per block
    shared_taps: bool
    description: str


CONFIGS = {
    "plain_cpu": Config("plain_cpu", 1, 64, 16, 5, "qam4", "rc", 0.5, True,
                        "64 blocks, K=16, M=5 (N=80), 4-QAM, RC roll-off 0.5"),
    "plain_gpu": Config("plain_gpu", 2, 4096, 128, 15, "qam16", "rrc", 0.1, True,
                        "4096 blocks, K=128, M=15 (N=1920), 16-QAM, RRC roll-off 0.1"),
    "ragged": Config("ragged", 3, 10000, None, None, "qam64", "rc", None, False,
                     "10000 blocks, K in {64..1024}, M in {3,5,7,9,15}, 64-QAM, "
                     "per-block RC with roll-off U[0.1, 0.9]"),
    "precision": Config("precision", 4, 2048, 1024, 15, "cn01", "rrc", 0.1, True,
                        "2048 blocks, K=1024, M=15 (N=15360), CN(0,1), RRC roll-off 0.1"),
    "differentiation": Config("differentiation", 5, 8192, 256, 9, "qam16", "rc", 0.3, True,
                              "8192 blocks, K=256, M=9 (N=2304), 16-QAM, trainable RC roll-off 0.3"),
}

RAGGED_K = (64, 128, 256, 512, 1024)
RAGGED_M = (3, 5, 7, 9, 15)


def _symbols(kind: str, rng, size):
    if kind.startswith("qam"):
        return qam(rng, int(kind[3:]), size)
    if kind == "cn01":
        return cn01(rng, size)
    raise ValueError(kind)


def _taps(kind: str, N: int, alpha: float) -> np.ndarray:
    if kind == "rc":
        return rc_taps(N, alpha)
    if kind == "rrc":
        return rrc_taps(N, alpha)
    raise ValueError(kind)


def make_uniform(cfg: Config | str, nblocks: Optional[int] = None):
    """(S complex64 [B, N], taps float32 [N]) for a uniform configuration.

    `nblocks` truncates the batch (the first blocks of the same seeded draw).
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if cfg.K is None:
        raise ValueError("ragged configuration: use make_ragged")
    N = cfg.K * cfg.M
    B = cfg.nblocks if nblocks is None else int(nblocks)
    r_sym, = rng_streams(cfg.seed, 1)
    S = _symbols(cfg.symbols, r_sym, (cfg.nblocks, N))[:B].astype(np.complex64)
    taps = _taps(cfg.taps, N, cfg.alpha).astype(np.float32)
    return np.ascontiguousarray(S), taps


@dataclasses.dataclass
class RaggedLayout:
    """Block table of a ragged batch: per block K, M, and element offsets."""
    K: np.ndarray          # int32 [B]
    M: np.ndarray          # int32 [B]
    x_off: np.ndarray      # int64 [B], complex elements
    tap_off: np.ndarray    # int64 [B], floats
    alpha: np.ndarray      # float64 [B] roll-off per block

    @property
    def N(self) -> np.ndarray:
        return self.K.astype(np.int64) * self.M.astype(np.int64)

    @property
    def total(self) -> int:
        return int(self.N.sum())

    def subset(self, idx) -> "RaggedLayout":
        """Layout of the blocks `idx`, re-packed contiguously."""
        idx = np.asarray(idx)
        K, M = self.K[idx], self.M[idx]
        N = K.astype(np.int64) * M
        off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
        return RaggedLayout(K.copy(), M.copy(), off, off.copy(), self.alpha[idx].copy())


def ragged_layout(seed: int, nblocks: int, Ks=RAGGED_K, Ms=RAGGED_M) -> RaggedLayout:
    r_k, r_m, r_a = rng_streams(seed, 4)[:3]
    K = np.asarray(Ks, dtype=np.int32)[r_k.integers(0, len(Ks), size=nblocks)]
    M = np.asarray(Ms, dtype=np.int32)[r_m.integers(0, len(Ms), size=nblocks)]
    alpha = r_a.uniform(0.1, 0.9, size=nblocks)
    N = K.astype(np.int64) * M
    off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
    return RaggedLayout(K, M, off, off.copy(), alpha)


def make_ragged(cfg: Config | str = "ragged", nblocks: Optional[int] = None):
    """(layout, S complex64 [sum N], taps float32 [sum N]) for the ragged batch.

    Every block has its own RC filter (roll-off from the layout), stored at the
    same offset as its coefficients.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    B = cfg.nblocks if nblocks is None else int(nblocks)
    lay = ragged_layout(cfg.seed, B)
    r_sym = rng_streams(cfg.seed, 4)[3]
    S = _symbols(cfg.symbols, r_sym, lay.total).astype(np.complex64)
    taps = np.empty(lay.total, dtype=np.float32)
    for b in range(B):
        N = int(lay.K[b]) * int(lay.M[b])
        o = int(lay.tap_off[b])
        taps[o:o + N] = _taps(cfg.taps, N, float(lay.alpha[b])).astype(np.float32)
    return lay, S, taps
