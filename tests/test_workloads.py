"""Seeded input generators (CPU only)."""
import math

import numpy as np

from paper_1604_06236_amd import workloads as W


def test_qam_levels_and_energy():
    rng = np.random.default_rng(0)
    for order in (4, 16, 64):
        x = W.qam(rng, order, 200000)
        L = int(math.sqrt(order))
        scale = math.sqrt(2 * (L * L - 1) / 3)
        lv = np.unique(np.round(x.real * scale).astype(int))
        assert list(lv) == list(range(-(L - 1), L, 2))
        assert abs(np.mean(np.abs(x) ** 2) - 1) < 0.02


def test_rc_and_rrc_taps():
    for N in (80, 1920, 2304):
        for alpha in (0.1, 0.3, 0.5, 0.9):
            rc = W.rc_taps(N, alpha)
            rrc = W.rrc_taps(N, alpha)
            assert abs(np.sum(rc ** 2) - 1) < 1e-12 and abs(np.sum(rrc ** 2) - 1) < 1e-12
            # flat top, symmetric, never below half the peak: always invertible
            assert np.allclose(rc[1:], rc[1:][::-1])
            assert rc.min() / rc.max() >= 0.5 - 1e-12
            assert rrc.min() / rrc.max() >= math.sqrt(0.5) - 1e-12
            assert np.allclose(rrc ** 2 / np.sum(rrc ** 2), rc / np.sum(rc))


def test_configs_are_seeded_and_shaped():
    S1, t1 = W.make_uniform("plain_cpu")
    S2, t2 = W.make_uniform("plain_cpu")
    assert S1.shape == (64, 80) and S1.dtype == np.complex64 and t1.dtype == np.float32
    assert np.array_equal(S1, S2) and np.array_equal(t1, t2)
    Sa, _ = W.make_uniform("plain_gpu", nblocks=10)
    assert Sa.shape == (10, 1920)


def test_ragged_layout():
    lay, S, taps = W.make_ragged("ragged", nblocks=300)
    assert set(np.unique(lay.K)) <= set(W.RAGGED_K)
    assert set(np.unique(lay.M)) <= set(W.RAGGED_M)
    assert lay.total == S.size == taps.size
    assert np.all(np.diff(lay.x_off) == lay.N[:-1])
    for b in (0, 7, 299):
        o, N = int(lay.tap_off[b]), int(lay.N[b])
        assert abs(np.sum(taps[o:o + N].astype(np.float64) ** 2) - 1) < 1e-5
    sub = lay.subset([3, 1])
    assert sub.x_off[0] == 0 and sub.x_off[1] == lay.N[3]
