"""The C-ABI library loads, exports every declared symbol, and validates
arguments on the host (no GPU needed: none of these calls reaches a launch)."""
import ctypes
import os
import re

import pytest

from paper_1604_06236_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "blocktransform.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(transform_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(nat.LIB_PATH):
        from paper_1604_06236_amd import build
        build.build(force=False)
    return nat.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
        assert n in nat.EXPORTED, n


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.transform_status_string(s).startswith(b"TF_")


def _fwd(lib, B, K, M, ts=0, compute=0, ptr=8):
    p = ctypes.c_void_p(ptr) if ptr else None
    q = ctypes.c_void_p(ptr + (1 << 30)) if ptr else None
    return lib.transform_forward(p, q, ctypes.c_void_p(ptr + (2 << 30)) if ptr else None, B, K, M,
                                 ts, compute, None, 0, None)


def test_host_validation(lib):
    assert _fwd(lib, 0, 16, 5, ptr=0) == nat.TF_OK                 # empty batch
    assert _fwd(lib, -1, 16, 5) == nat.TF_EINVAL
    for K, M in ((3, 5), (2048, 1), (0, 4), (16, 0), (16, 17)):
        assert _fwd(lib, 4, K, M) == nat.TF_EUNSUPPORTED, (K, M)
    assert _fwd(lib, 4, 16, 5, ptr=0) == nat.TF_EINVAL              # null pointers
    assert _fwd(lib, 4, 16, 5, ts=7) == nat.TF_EINVAL               # tap stride not 0 or N
    assert _fwd(lib, 4, 16, 5, ptr=12) == nat.TF_EINVAL             # misaligned complex pointer
    assert _fwd(lib, 4, 16, 5, compute=9) == nat.TF_EUNSUPPORTED
    # overlapping input and output
    p = ctypes.c_void_p(1 << 20)
    t = ctypes.c_void_p(1 << 32)
    assert lib.transform_forward(p, t, ctypes.c_void_p((1 << 20) + 64), 4, 16, 5, 0, 0, None, 0,
                                 None) == nat.TF_EINVAL
    # the tap gradient needs the coefficients
    assert lib.transform_adjoint(ctypes.c_void_p(1 << 20), t, None, ctypes.c_void_p(1 << 31),
                                 ctypes.c_void_p(1 << 33), 4, 16, 5, 0, 0, None, 0,
                                 None) == nat.TF_EINVAL


@pytest.mark.parametrize("compute", [nat.TF_SPLIT_BF16, nat.TF_SPLIT_FP16])
def test_host_validation_split_modes(lib, compute):
    """The split-precision modes run the same argument checks before any launch."""
    K, M = 1024, 15
    assert _fwd(lib, 4, K, M, compute=compute, ptr=0) == nat.TF_EINVAL       # null pointers
    assert _fwd(lib, 4, K, M, ts=7, compute=compute) == nat.TF_EINVAL        # tap stride
    assert _fwd(lib, -1, K, M, compute=compute) == nat.TF_EINVAL             # negative count
    assert _fwd(lib, 4, K, M, ptr=12, compute=compute) == nat.TF_EINVAL      # misaligned
    p = ctypes.c_void_p(1 << 20)
    t = ctypes.c_void_p(1 << 32)
    assert lib.transform_forward(p, t, p, 4, K, M, 0, compute, None, 0, None) == nat.TF_EINVAL
    assert lib.transform_adjoint(p, t, None, ctypes.c_void_p((1 << 20) + 64), None, 4, K, M, 0,
                                 compute, None, 0, None) == nat.TF_EINVAL
    # a size the split path does not cover stays unsupported once the arguments are valid
    assert _fwd(lib, 4, 128, 15, compute=compute) == nat.TF_EUNSUPPORTED
    assert _fwd(lib, 0, K, M, compute=compute, ptr=0) == nat.TF_OK           # empty batch


def test_schedule_registry(lib, tmp_path):
    from paper_1604_06236_amd import transform as T
    for K in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024):
        for M in range(1, 17):
            sch = T.schedules(K, M)
            assert sch, (K, M)
            for s in sch:
                prod = 1
                for r in s["radices"]:
                    prod *= r
                assert prod == K * M and s["lds_bytes"] <= 160 * 1024
    assert lib.transform_schedule_count(3, 3) == 0
    assert lib.transform_schedule_select(128, 15, 99, 0) == nat.TF_EINVAL
    assert lib.transform_schedule_select(128, 15, 1, 512) == nat.TF_OK
    path = str(tmp_path / "sched.json").encode()
    assert lib.transform_save_schedule(path) == nat.TF_OK
    assert lib.transform_schedule_select(128, 15, -1, 0) == nat.TF_OK
    assert lib.transform_load_schedule(path) == nat.TF_OK
    txt = open(path.decode()).read()
    assert '"128,15": [-1, 0]' in txt or '"128,15"' in txt
    assert lib.transform_schedule_select(128, 15, -1, 0) == nat.TF_OK


def test_package_schedules_load_as_written(lib):
    """The library's loader applies exactly the fused "K,M": [schedule, grid cap] entries of
    the package's schedules.json; the other keys (the ragged kernel's options) leave every
    other shape's selection alone."""
    import ctypes
    import json
    import os
    path = os.path.join(os.path.dirname(nat.__file__), "schedules.json")
    sel = json.load(open(path))
    fused = {tuple(int(v) for v in k.split(",")): v for k, v in sel.items() if "," in k}
    assert fused and all(isinstance(v, list) and len(v) == 2 for v in fused.values())
    shapes = [(K, M) for K in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024) for M in range(1, 17)]
    i, c = ctypes.c_int32(), ctypes.c_int32()

    def selected(K, M):
        assert lib.transform_schedule_selected(K, M, ctypes.byref(i), ctypes.byref(c)) == nat.TF_OK
        return [i.value, c.value]
    for K, M in shapes:
        assert lib.transform_schedule_select(K, M, -1, 0) == nat.TF_OK
    before = {km: selected(*km) for km in shapes}
    assert lib.transform_load_schedule(path.encode()) == nat.TF_OK
    for km in shapes:
        assert selected(*km) == (fused[km] if km in fused else before[km]), km


def test_ragged_prefetch_registry(lib):
    """Per-class tile-pipelining choices of the ragged kernel: host-side table only."""
    import ctypes
    v = ctypes.c_int32(-7)
    sel = lambda K, M, b: (lib.transform_ragged_prefetch_selected(K, M, b, ctypes.byref(v)), v.value)
    assert lib.transform_ragged_prefetch_select(128, 15, 3, 0) == nat.TF_EINVAL       # body
    assert lib.transform_ragged_prefetch_select(128, 15, 0, 2) == nat.TF_EINVAL       # value
    assert lib.transform_ragged_prefetch_select(32, 15, 0, 0) == nat.TF_EUNSUPPORTED  # no such class
    assert lib.transform_ragged_prefetch_selected(128, 15, 0, None) == nat.TF_EINVAL
    # the (1024, 15) half-block body has no prefetching form
    assert sel(1024, 15, 0) == (nat.TF_OK, 0)
    assert lib.transform_ragged_prefetch_select(1024, 15, 0, 1) == nat.TF_EUNSUPPORTED
    # (128, 15) forward prefetches by default; off, then back to the default
    assert lib.transform_ragged_prefetch_select(128, 15, 0, -1) == nat.TF_OK
    assert sel(128, 15, 0) == (nat.TF_OK, 1)
    assert lib.transform_ragged_prefetch_select(128, 15, 0, 0) == nat.TF_OK
    assert sel(128, 15, 0) == (nat.TF_OK, 0)
    assert sel(128, 15, 1) == (nat.TF_OK, 1)                  # other bodies untouched
    assert lib.transform_ragged_prefetch_select(128, 15, 0, 1) == nat.TF_OK
    assert sel(128, 15, 0) == (nat.TF_OK, 1)
    # (128, 15) with the tap gradient has no prefetching form (it would spill)
    assert sel(128, 15, 2) == (nat.TF_OK, 0)
    assert lib.transform_ragged_prefetch_select(128, 15, 2, 1) == nat.TF_EUNSUPPORTED
    assert lib.transform_ragged_prefetch_select(128, 15, 2, 0) == nat.TF_OK


def test_workspace_sizes_host_only(lib):
    assert lib.transform_workspace_size(10, 16, 5, 0, 0, 0) == 0
    # plain path: two complex buffers, plus tap-gradient rows when shared
    assert lib.transform_workspace_size(10, 16, 5, 0, 3, 0) == 2 * 10 * 80 * 8
    assert lib.transform_workspace_size(10, 16, 5, 0, 3, 1) == 2 * 10 * 80 * 8 + 10 * 80 * 4
    assert lib.transform_workspace_size(0, 16, 5, 0, 3, 1) == 0
    # more than one 16-row chunk: the partial rows plus one row of chunk sums per chunk
    assert lib.transform_workspace_size(100, 16, 5, 0, 3, 1) == 2 * 100 * 80 * 8 + (100 + 7) * 80 * 4
    assert lib.transform_workspace_size(16, 16, 5, 0, 3, 1) == 2 * 16 * 80 * 8 + 16 * 80 * 4
    assert lib.transform_workspace_size(17, 16, 5, 0, 3, 1) == 2 * 17 * 80 * 8 + (17 + 2) * 80 * 4


def test_adjacent_buffers_are_not_overlap(lib):
    """taps_bar placed right after samples_bar is legal: validation must pass it on
    (on a machine without a GPU the call then fails in the runtime, not in validation)."""
    B, K, M = 4, 16, 5
    N = K * M
    yb = 1 << 20
    tb = yb + B * N * 8                      # immediately after samples_bar
    rc = lib.transform_adjoint(ctypes.c_void_p(yb), ctypes.c_void_p(1 << 32),
                               ctypes.c_void_p(1 << 34), ctypes.c_void_p(1 << 36),
                               ctypes.c_void_p(tb), B, K, M, 0, 0, None, 0, None)
    assert rc != nat.TF_EINVAL
    rc = lib.transform_adjoint(ctypes.c_void_p(yb), ctypes.c_void_p(1 << 32),
                               ctypes.c_void_p(1 << 34), ctypes.c_void_p(1 << 36),
                               ctypes.c_void_p(tb - 8), B, K, M, 0, 0, None, 0, None)
    assert rc == nat.TF_EINVAL


def test_nufft_host_validation(lib):
    """Argument checks of the type-4/5 and NFFT entry points, all before any launch."""
    vp = ctypes.c_void_p
    t, x, y, ws = vp(1 << 20), vp(1 << 30), vp(1 << 31), vp(1 << 33)
    big = 1 << 30
    # empty batches are no-ops
    assert lib.nufft_type5(None, None, None, 0, 64, 6, 0.01, None, 0, None) == nat.TF_OK
    assert lib.nufft_solve(4, 3, None, None, None, 0, 64, 2, 0.01, None, 0, None) == nat.TF_OK
    # shapes
    assert lib.nufft_type5(t, x, y, 1, 48, 6, 0.01, ws, big, None) == nat.TF_EUNSUPPORTED
    assert lib.nufft_type5(t, x, y, 1, 2048, 6, 0.01, ws, big, None) == nat.TF_EUNSUPPORTED
    assert lib.nufft_type4(t, x, y, 1, 64, 0, 0.01, ws, big, None) == nat.TF_EUNSUPPORTED
    assert lib.nufft_solve(5, 2, t, x, y, 1, 1024, 15, 0.01, ws, big, None) == nat.TF_EUNSUPPORTED
    # damping, options, type
    assert lib.nufft_type5(t, x, y, 1, 64, 6, 0.0, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_type5(t, x, y, 1, 64, 6, float("nan"), ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_solve(5, 4, t, x, y, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_solve(3, 0, t, x, y, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    # workspace, pointers, overlaps
    need = lib.nufft_workspace_size(1, 64, 6)
    assert need > 0 and lib.nufft_workspace_size_ex(1, 64, 6, 2) > need
    assert lib.nufft_type5(t, x, y, 1, 64, 6, 0.01, ws, need - 1, None) == nat.TF_EWORKSPACE
    assert lib.nufft_type5(t, x, y, 1, 64, 6, 0.01, vp((1 << 33) + 8), big, None) == nat.TF_EWORKSPACE
    assert lib.nufft_type5(None, x, y, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_type4_refined(t, x, x, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_type5(t, x, ws, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    # setup once, apply many: the setup needs no input or output, the application does
    assert lib.nufft_setup(0, None, 0, 64, 6, 0.01, None, 0, None) == nat.TF_OK
    assert lib.nufft_setup(0, None, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_setup(0, t, 1, 64, 6, 0.01, ws, need - 1, None) == nat.TF_EWORKSPACE
    assert lib.nufft_setup(8, t, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_setup(0, vp(1 << 33), 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL   # t inside ws
    assert lib.nufft_apply(3, 0, t, x, y, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_apply(5, 0, t, None, y, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_apply(4, 1, t, x, x, 1, 64, 6, 0.01, ws, big, None) == nat.TF_EINVAL
    assert lib.nufft_apply(5, 0, t, x, y, 1, 2048, 6, 0.01, ws, big, None) == nat.TF_EUNSUPPORTED
    # sums
    assert lib.nudft_type1(t, x, y, 1, 65537, 64, None) == nat.TF_EUNSUPPORTED
    assert lib.nudft_type2(t, x, y, 1, 64, 0, None) == nat.TF_EUNSUPPORTED
    assert lib.nfft_workspace_size(1, 1000) == 0 and lib.nfft_workspace_size(1, 6144) > 0
    assert lib.nfft_type1(t, x, y, 1, 64, 1000, ws, big, None) == nat.TF_EUNSUPPORTED
