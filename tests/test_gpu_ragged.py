"""GPU parity of the ragged kernel (one launch per direction, HIP graph) against the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_06236_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a, np.complex128) - b).ravel()) / np.linalg.norm(b.ravel()))


def per_block_max(a, b, lay):
    worst = 0.0
    for o, n in zip(lay.x_off, lay.N):
        sl = slice(int(o), int(o + n))
        worst = max(worst, float(np.linalg.norm(a[sl] - b[sl]) / np.linalg.norm(b[sl])))
    return worst


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_1604_06236_amd import transform
    return transform


@pytest.mark.parametrize("use_graph", [False, True])
def test_ragged_forward_inverse_adjoint(T, use_graph):
    lay, S, taps = W.make_ragged("ragged", nblocks=260)      # every (K, M) class, ragged tail
    print(f"case ragged blocks=260 graph={use_graph}", flush=True)
    plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
    y_ref = O.forward_ragged(lay.N, lay.x_off, lay.tap_off, S, taps)
    dS, dt = _dev(S), _dev(taps)
    y = plan.execute("forward", dS, dt, use_graph=use_graph)
    yh = _host(y)
    assert rel_l2(yh, y_ref) < TOL and per_block_max(yh, y_ref, lay) < TOL
    back = _host(plan.execute("inverse", y, dt, use_graph=use_graph))
    assert rel_l2(back, S.astype(np.complex128)) < TOL
    yb = W.cn01(np.random.default_rng(4), lay.total).astype(np.complex64)
    inv_ref = O.inverse_ragged(lay.N, lay.x_off, lay.tap_off, yb, taps)
    inv = _host(plan.execute("inverse", _dev(yb), dt, use_graph=use_graph))
    assert rel_l2(inv, inv_ref) < TOL and per_block_max(inv, inv_ref, lay) < TOL
    sb_ref, tb_ref = O.adjoint_ragged(lay.N, lay.x_off, lay.tap_off, yb, taps, S)
    sb, tb = plan.execute("adjoint", _dev(yb), dt, aux=dS, want_taps_bar=True, use_graph=use_graph)
    assert rel_l2(_host(sb), sb_ref) < TOL
    tbh = _host(tb).astype(np.float64)
    assert float(np.linalg.norm(tbh - tb_ref) / np.linalg.norm(tb_ref)) < TOL
    sb2 = plan.execute("adjoint", _dev(yb), dt, use_graph=use_graph)
    assert rel_l2(_host(sb2), sb_ref) < TOL
    plan.close()


def test_ragged_graph_replays_match_eager(T):
    """A captured graph replayed several times, with other work in between, gives
    the eager result every time."""
    import torch
    lay, S, taps = W.make_ragged("ragged", nblocks=120)
    plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
    dS, dt = _dev(S), _dev(taps)
    eager = _host(plan.execute("forward", dS, dt, use_graph=False))
    out = torch.empty_like(dS)
    for rep in range(4):
        out.zero_()
        plan.execute("forward", dS, dt, out=out, use_graph=True)
        got = _host(out)
        assert np.array_equal(got.view(np.uint64), eager.view(np.uint64)), rep
        _ = (dS * 2).sum()          # unrelated eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_ragged_unsorted_offsets_and_gaps(T):
    """Blocks listed out of memory order, with unused gaps between them."""
    rng = np.random.default_rng(11)
    Ks = rng.choice([64, 256, 1024], size=9).astype(np.int32)
    Ms = rng.choice([3, 9, 15], size=9).astype(np.int32)
    N = Ks.astype(np.int64) * Ms
    perm = rng.permutation(9)
    off = np.zeros(9, np.int64)
    pos = 0
    for b in perm:
        pos += 16                          # gap
        off[b] = pos
        pos += N[b]
    total = int(pos + 16)
    S = W.qam(rng, 64, total).astype(np.complex64)
    taps = np.ones(total, np.float32)
    for b in range(9):
        taps[off[b]:off[b] + N[b]] = W.rc_taps(int(N[b]), 0.4)
    plan = T.RaggedPlan(Ks, Ms, off, off, total)
    out = _dev(np.zeros(total, np.complex64))
    y = _host(plan.execute("forward", _dev(S), _dev(taps), out=out))
    ref = O.forward_ragged(N, off, off, S, taps)
    for b in range(9):
        sl = slice(int(off[b]), int(off[b] + N[b]))
        assert rel_l2(y[sl], ref[sl]) < TOL
    # gaps untouched
    mask = np.ones(total, bool)
    for b in range(9):
        mask[off[b]:off[b] + N[b]] = False
    assert np.all(y[mask] == 0)
    plan.close()


def test_ragged_full_batch(T):
    """The full 10,000-block batch in the benchmark's launch (HIP graph replay), every block of
    every direction against the FFT form of the oracle, 40 seeded blocks against the O(N^2)
    sums, and every block through the inverse round trip."""
    from oracle import fftref as F
    lay, S, taps = W.make_ragged("ragged")
    print(f"case ragged full blocks={lay.K.size} points={lay.total}", flush=True)
    args = (lay.N, lay.x_off, lay.tap_off)
    yb = W.cn01(W.rng_streams(W.CONFIGS["ragged"].seed + 100, 1)[0], lay.total).astype(np.complex64)
    plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
    dS, dt, dyb = _dev(S), _dev(taps), _dev(yb)
    y = plan.execute("forward", dS, dt, use_graph=True)
    yh = _host(y)
    inv = _host(plan.execute("inverse", dyb, dt, use_graph=True))
    sb, tb = plan.execute("adjoint", dyb, dt, aux=dS, want_taps_bar=True, use_graph=True)
    sb, tb = _host(sb), _host(tb).astype(np.float64)
    sb2 = _host(plan.execute("adjoint", dyb, dt, use_graph=True))
    back = _host(plan.execute("inverse", y, dt, use_graph=True))
    y_ref = F.forward_ragged(*args, S, taps)
    inv_ref = F.inverse_ragged(*args, yb, taps)
    sb_ref, tb_ref = F.adjoint_ragged(*args, yb, taps, S)
    for got, ref in ((yh, y_ref), (inv, inv_ref), (sb, sb_ref), (sb2, sb_ref)):
        assert rel_l2(got, ref) < TOL and per_block_max(got, ref, lay) < TOL
    assert float(np.linalg.norm(tb - tb_ref) / np.linalg.norm(tb_ref)) < TOL
    assert rel_l2(back, S.astype(np.complex128)) < TOL and per_block_max(back, S.astype(np.complex128), lay) < TOL
    # a seeded sample against the O(N^2) sums
    idx = np.sort(np.random.default_rng(1).choice(lay.K.size, 40, replace=False))
    sub = lay.subset(idx)

    def pick(x):
        return np.concatenate([x[int(lay.x_off[b]):int(lay.x_off[b] + lay.N[b])] for b in idx])
    tsub = np.concatenate([taps[int(lay.tap_off[b]):int(lay.tap_off[b] + lay.N[b])] for b in idx])
    sargs = (sub.N, sub.x_off, sub.tap_off)
    assert rel_l2(pick(yh), O.forward_ragged(*sargs, pick(S), tsub)) < TOL
    assert rel_l2(pick(inv), O.inverse_ragged(*sargs, pick(yb), tsub)) < TOL
    assert rel_l2(pick(sb), O.adjoint_ragged(*sargs, pick(yb), tsub)[0]) < TOL
    plan.close()


def test_ragged_plan_rejects_bad_layouts(T):
    from paper_1604_06236_amd._native import TransformError
    with pytest.raises(TransformError):
        T.RaggedPlan([48], [3], [0], [0], 144)          # K not a power of two
    with pytest.raises(TransformError):
        T.RaggedPlan([64], [3], [100], [0], 200)        # block runs past the end


def test_ragged_chunk_sizes_agree(T):
    """Work-item sizes only change which workgroup runs a tile, never the arithmetic:
    every chunking gives bit-identical results."""
    lay, S, taps = W.make_ragged("ragged", nblocks=400)
    dS, dt = _dev(S), _dev(taps)
    outs = []
    for chunk in (1, 3, 4, 16):
        plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total, chunk_tiles=chunk)
        outs.append(_host(plan.execute("forward", dS, dt, use_graph=False)))
        plan.close()
    for o in outs[1:]:
        assert np.array_equal(o.view(np.uint64), outs[0].view(np.uint64))


def test_ragged_prefetch_choices_agree(T):
    """The per-class tile pipelining (prefetch of the next tile on or off, chosen by the
    autotuner) only moves loads in time: forward, inverse, adjoint and the tap-gradient adjoint
    match the oracle either way, and agree with each other to rounding (the two forms of a body
    are compiled separately, so the compiler may contract different multiply-adds)."""
    lay, S, taps = W.make_ragged("ragged", nblocks=600)      # several tiles per item per class
    dS, dt = _dev(S), _dev(taps)
    yb = W.cn01(np.random.default_rng(9), lay.total).astype(np.complex64)
    dyb = _dev(yb)
    classes = sorted(set(zip(lay.K.tolist(), lay.M.tolist())))
    print(f"case ragged prefetch choices, blocks=600, classes={len(classes)}", flush=True)

    def run():
        plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total, chunk_tiles=4)
        y = _host(plan.execute("forward", dS, dt, use_graph=False))
        inv = _host(plan.execute("inverse", dyb, dt, use_graph=False))
        sb, tb = plan.execute("adjoint", dyb, dt, aux=dS, want_taps_bar=True, use_graph=False)
        sb0 = _host(plan.execute("adjoint", dyb, dt, use_graph=False))
        out = (y, inv, _host(sb), _host(tb), sb0)
        plan.close()
        return out

    try:
        for K, M in classes:
            for b in range(3):
                T.ragged_prefetch_select(K, M, b, -1)
        assert any(T.ragged_prefetch_selected(K, M, b) for K, M in classes for b in range(3))
        ref = run()
        for K, M in classes:
            for b in range(3):
                T.ragged_prefetch_select(K, M, b, 0)
        off = run()
    finally:
        for K, M in classes:
            for b in range(3):
                T.ragged_prefetch_select(K, M, b, -1)
        T.load_schedules()
    y_ref = O.forward_ragged(lay.N, lay.x_off, lay.tap_off, S, taps)
    inv_ref = O.inverse_ragged(lay.N, lay.x_off, lay.tap_off, yb, taps)
    sb_ref, tb_ref = O.adjoint_ragged(lay.N, lay.x_off, lay.tap_off, yb, taps, S)
    for out in (ref, off):
        y, inv, sb, tb, sb0 = out
        assert rel_l2(y, y_ref) < TOL and per_block_max(y, y_ref, lay) < TOL
        assert rel_l2(inv, inv_ref) < TOL and per_block_max(inv, inv_ref, lay) < TOL
        assert rel_l2(sb, sb_ref) < TOL and rel_l2(sb0, sb_ref) < TOL
        assert rel_l2(tb, tb_ref) < TOL
    for a, b in zip(ref, off):
        assert rel_l2(a, b.astype(np.complex128)) < 1e-6


def test_ragged_plan_on_two_streams(T):
    """One plan executed on two streams at once (forward on one, adjoint on the other, eager
    and graph-replayed): a launch keeps no state in the plan's device memory, so both
    directions' outputs are exact (bit-identical to a lone execution)."""
    import torch
    lay, S, taps = W.make_ragged("ragged", nblocks=200)
    plan = T.RaggedPlan(lay.K, lay.M, lay.x_off, lay.tap_off, lay.total)
    dS, dt = _dev(S), _dev(taps)
    yb = _dev(W.cn01(np.random.default_rng(6), lay.total).astype(np.complex64))
    y_lone = _host(plan.execute("forward", dS, dt, use_graph=False))
    sb_lone = _host(plan.execute("adjoint", yb, dt, use_graph=False))
    assert rel_l2(y_lone, O.forward_ragged(lay.N, lay.x_off, lay.tap_off, S, taps)) < TOL
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for use_graph in (False, True):
        ys = [torch.empty_like(dS) for _ in range(6)]
        sbs = [torch.empty_like(dS) for _ in range(6)]
        for i in range(6):
            with torch.cuda.stream(s1):
                plan.execute("forward", dS, dt, out=ys[i], use_graph=use_graph)
            with torch.cuda.stream(s2):
                plan.execute("adjoint", yb, dt, out=sbs[i], use_graph=use_graph)
        torch.cuda.synchronize()
        for i in range(6):
            assert np.array_equal(_host(ys[i]).view(np.uint64), y_lone.view(np.uint64)), (use_graph, i)
            assert np.array_equal(_host(sbs[i]).view(np.uint64), sb_lone.view(np.uint64)), (use_graph, i)
    plan.close()
