// C ABI of the block-transform library: argument validation, schedule
// registry and selection, per-device plan tables, and dispatch to the fused,
// plain and ragged kernels.  Host code only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"
#include "bt_fused.hpp"
#include "bt_plain.hpp"

namespace bt {
void register_fused_m01_04(std::vector<FusedEntry> &v);
void register_fused_m05_08(std::vector<FusedEntry> &v);
void register_fused_m09_12(std::vector<FusedEntry> &v);
void register_fused_m13_16(std::vector<FusedEntry> &v);
void register_fused_tuned(std::vector<FusedEntry> &v);
void register_fused_half(std::vector<FusedEntry> &v);

thread_local std::string g_last_error;

void set_error(const char *what, hipError_t e)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
}

// ------------------------------------------------------------------ registry
struct Registry {
    std::vector<FusedEntry> entries;
    std::map<std::pair<int, int>, std::vector<int>> by_km;   // first index = default schedule
};

static Registry &registry()
{
    static Registry *r = [] {
        Registry *g = new Registry;
        register_fused_m01_04(g->entries);
        register_fused_m05_08(g->entries);
        register_fused_m09_12(g->entries);
        register_fused_m13_16(g->entries);
        register_fused_tuned(g->entries);
        register_fused_half(g->entries);
        for (int i = 0; i < (int)g->entries.size(); ++i)
            g->by_km[{g->entries[i].K, g->entries[i].M}].push_back(i);
        return g;
    }();
    return *r;
}

struct Selection {
    int idx = -1;       // index into by_km list; -1 = default
    int grid_cap = 0;
};

static std::mutex g_mu;
static std::map<std::pair<int, int>, Selection> g_select;

struct DeviceState {
    int cus = 0;
    std::map<int, c32 *> tw;                       // entry -> twiddle table
    std::map<std::pair<int, int>, int> occ;        // (entry, kernel variant) -> workgroups per CU
    std::map<std::pair<int, int>, c32 *> roots;    // (K, M) -> N-th roots (plain path)
    float *scratch = nullptr;                      // this device's copy of the no-alloc scratch array
};
static std::map<int, DeviceState> g_dev;

bool supported_km(int K, int M)
{
    if (K < 1 || K > 1024 || (K & (K - 1)) != 0) return false;
    if (M < 1 || M > 16) return false;
    return true;
}

static int current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) {
        set_error("hipGetDevice", e);
        return TF_EHIP;
    }
    return TF_OK;
}

static DeviceState &dev_state(int dev)
{
    DeviceState &d = g_dev[dev];
    if (d.cus == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        d.cus = cus;
    }
    return d;
}

// entry chosen for (K, M), honouring the selection table
static int chosen_entry(int K, int M, int *grid_cap)
{
    Registry &r = registry();
    auto it = r.by_km.find({K, M});
    if (it == r.by_km.end()) return -1;
    int pos = 0;
    *grid_cap = 0;
    auto s = g_select.find({K, M});
    if (s != g_select.end()) {
        if (s->second.idx >= 0 && s->second.idx < (int)it->second.size()) pos = s->second.idx;
        *grid_cap = s->second.grid_cap;
    }
    return it->second[pos];
}

// base twiddles: for pass p >= 1 with stride Ns and radix R, entry [jm] =
// e^{+j 2 pi jm / (Ns R)} for jm < Ns, computed in double and rounded once
static std::vector<c32> build_twiddles(const FusedEntry &e)
{
    std::vector<c32> t;
    t.reserve(e.tw_entries);
    long ns = e.radix[0];
    for (int p = 1; p < e.npass; ++p) {
        const long R = e.radix[p];
        const long L = ns * R;
        for (long jm = 0; jm < ns; ++jm) {
            const double ang = 2.0 * M_PI * double(jm) / double(L);
            t.push_back(c32{float(std::cos(ang)), float(std::sin(ang))});
        }
        ns *= R;
    }
    return t;
}

static int upload(const std::vector<c32> &h, c32 **out)
{
    c32 *d = nullptr;
    size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(c32);
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) {
        set_error("hipMalloc(table)", e);
        return TF_EHIP;
    }
    if (!h.empty()) {
        e = hipMemcpy(d, h.data(), h.size() * sizeof(c32), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            set_error("hipMemcpy(table)", e);
            hipFree(d);
            return TF_EHIP;
        }
    }
    *out = d;
    return TF_OK;
}

// twiddle table of an entry and occupancy of one of its kernels on the current
// device (built once)
static int entry_tables(int dev, int idx, int side, int tg, const c32 **tw, int *occ)
{
    DeviceState &d = dev_state(dev);
    const FusedEntry &e = registry().entries[idx];
    auto it = d.tw.find(idx);
    if (it == d.tw.end()) {
        c32 *p = nullptr;
        int rc = upload(build_twiddles(e), &p);
        if (rc) return rc;
        it = d.tw.emplace(idx, p).first;
    }
    const int variant = side * 2 + (tg ? 1 : 0);
    auto oc = d.occ.find({idx, variant});
    if (oc == d.occ.end()) {
        int n = 0;
        hipError_t he = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, reinterpret_cast<const void *>(e.kernel[side][tg ? 1 : 0]), e.TB * e.BPW, 0);
        oc = d.occ.emplace(std::make_pair(idx, variant), (he == hipSuccess && n > 0) ? n : 1).first;
    }
    *tw = it->second;
    *occ = oc->second;
    return TF_OK;
}

static int plain_roots(int dev, int K, int M, const c32 **roots)
{
    DeviceState &d = dev_state(dev);
    auto it = d.roots.find({K, M});
    if (it == d.roots.end()) {
        const long N = long(K) * M;
        std::vector<c32> h(N);
        for (long k = 0; k < N; ++k) {
            const double ang = 2.0 * M_PI * double(k) / double(N);
            h[k] = c32{float(std::cos(ang)), float(std::sin(ang))};
        }
        c32 *p = nullptr;
        int rc = upload(h, &p);
        if (rc) return rc;
        it = d.roots.emplace(std::make_pair(K, M), p).first;
    }
    *roots = it->second;
    return TF_OK;
}

// ------------------------------------------------------------------ launch geometry
struct Geometry {
    int idx;
    unsigned grid;
    int64_t rows;        // partial tap-gradient rows (grid * BPW)
};

static size_t fused_ws_bytes(int64_t rows, int64_t N)
{
    const int64_t nch = rows_reduce_chunks(rows);
    return size_t(rows + (nch > 1 ? nch : 0)) * N * sizeof(float);
}

// ws_cap: when nonzero, the grid is also capped so that the shared tap gradient's
// partial rows and chunk sums fit in ws_cap bytes
static int fused_geometry(int dev, int K, int M, int64_t nblocks, int side, bool tg,
                          bool shared_tapgrad, Geometry *g, const c32 **tw, size_t ws_cap = 0)
{
    int cap = 0;
    int idx = chosen_entry(K, M, &cap);
    if (idx < 0) return TF_EUNSUPPORTED;
    int occ = 1;
    int rc = entry_tables(dev, idx, side, tg, tw, &occ);
    if (rc) return rc;
    const FusedEntry &e = registry().entries[idx];
    const int64_t groups = (nblocks + e.BPW - 1) / e.BPW;
    int64_t grid = groups;
    const int64_t resident = int64_t(occ) * dev_state(dev).cus;
    if (shared_tapgrad && grid > resident) grid = resident;   // bound the partial rows
    if (cap > 0 && grid > cap) grid = cap;
    if (grid > 0x7fffffff) grid = 0x7fffffff;
    if (grid < 1) grid = 1;
    if (shared_tapgrad && ws_cap > 0) {
        const int64_t N = int64_t(K) * M;
        while (grid > 1 && fused_ws_bytes(grid * e.BPW, N) > ws_cap) grid = (grid + 1) / 2;
        if (fused_ws_bytes(grid * e.BPW, N) > ws_cap) return TF_EWORKSPACE;
    }
    g->idx = idx;
    g->grid = unsigned(grid);
    g->rows = grid * e.BPW;
    return TF_OK;
}

} // namespace bt

using namespace bt;

// ------------------------------------------------------------------ validation helpers
static bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// [a, a + abytes) and [b, b + bbytes) intersect
static bool overlap2(const void *a, size_t abytes, const void *b, size_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bbytes && y < x + abytes;
}

static bool overlap(const void *a, const void *b, size_t bytes) { return overlap2(a, bytes, b, bytes); }

static int check_common(const void *in, const float *taps, const void *out, int64_t nblocks,
                        int32_t K, int32_t M, int64_t tap_stride, int32_t compute)
{
    if (!supported_km(K, M)) return TF_EUNSUPPORTED;
    const bool split = compute == TF_SPLIT_BF16 || compute == TF_SPLIT_FP16;
    if (compute != TF_FP32 && compute != TF_PLAIN_FP32 && !split) return TF_EUNSUPPORTED;
    // argument checks first, for every compute mode: no launch sees a bad pointer or size
    if (nblocks < 0) return TF_EINVAL;
    const int64_t N = int64_t(K) * M;
    if (tap_stride != 0 && tap_stride != N) return TF_EINVAL;
    if (nblocks > 0) {
        if (!in || !out || !taps) return TF_EINVAL;
        if (!aligned(in, 8) || !aligned(out, 8) || !aligned(taps, 4)) return TF_EINVAL;
        if (overlap(in, out, size_t(nblocks) * N * 8)) return TF_EINVAL;
    }
    if (split) return split_supported(K, M, compute);
    return TF_OK;
}

static size_t plain_ws_bytes(int64_t nblocks, int64_t N, bool tapgrad, bool shared)
{
    size_t b = size_t(2) * nblocks * N * sizeof(c32);
    if (tapgrad && shared) {
        const int64_t nch = rows_reduce_chunks(nblocks);
        b += size_t(nblocks + (nch > 1 ? nch : 0)) * N * sizeof(float);
    }
    return b;
}

extern "C" size_t transform_workspace_size(int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                                           int32_t compute, int32_t with_tapbar)
{
    if (!supported_km(K, M) || nblocks <= 0) return 0;
    const int64_t N = int64_t(K) * M;
    const bool shared = tap_stride == 0;
    if (compute == TF_PLAIN_FP32) return plain_ws_bytes(nblocks, N, with_tapbar != 0, shared);
    if (compute == TF_SPLIT_BF16 || compute == TF_SPLIT_FP16)
        return split_workspace_size(nblocks, K, M, tap_stride, compute, with_tapbar);
    if (!(with_tapbar && shared)) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    if (current_device(&dev)) return 0;
    // large enough for either tap-gradient kernel (their occupancies may differ)
    size_t need = 0;
    for (int side : {int(SIDE_IN), int(SIDE_OUT)}) {
        Geometry g{};
        const c32 *tw = nullptr;
        if (fused_geometry(dev, K, M, nblocks, side, true, true, &g, &tw)) return 0;
        need = std::max(need, fused_ws_bytes(g.rows, N));
    }
    return need;
}

// One fused or plain run.  side: where the filter applies (SIDE_IN: positive
// exponent; SIDE_OUT: negative exponent); div: divide by N Lambda instead of
// multiplying by Lambda; tg: also compute the tap gradient into taps_bar.
static int run(const void *in, const float *taps, void *out, const void *aux, float *taps_bar,
               int32_t *status, int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
               int32_t compute, int side, int div, bool tg, void *ws, size_t ws_bytes, void *stream,
               bool ws_caps_grid = false)
{
    const int64_t N = int64_t(K) * M;
    const bool shared = tap_stride == 0;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    // The lock covers the lookups in the shared caches only (schedule choice, per-device
    // tables, occupancies); what they hand out lives until the process ends, so the launches
    // themselves run unlocked and calls from several threads or streams do not serialise.

    if (compute == TF_PLAIN_FP32) {
        if (tg && side == SIDE_IN) return TF_EUNSUPPORTED;
        const size_t need = plain_ws_bytes(nblocks, N, tg, shared);
        if (!ws || ws_bytes < need || !aligned(ws, 8)) return TF_EWORKSPACE;
        const c32 *roots = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            rc = plain_roots(dev, K, M, &roots);
        }
        if (rc) return rc;
        c32 *ws0 = reinterpret_cast<c32 *>(ws);
        c32 *ws1 = ws0 + nblocks * N;
        float *part = reinterpret_cast<float *>(ws1 + nblocks * N);
        PlainArgs a{};
        a.K = K;
        a.M = M;
        a.nblocks = nblocks;
        a.tap_stride = tap_stride;
        a.taps = taps;
        a.roots = roots;
        a.aux = reinterpret_cast<const c32 *>(aux);
        a.out = reinterpret_cast<c32 *>(out);
        a.status = status;
        a.conj_io = side == SIDE_OUT;
        a.in_op = side == SIDE_IN ? (div ? IN_DIV_NTAP : IN_MUL_TAP) : IN_NONE;
        a.out_op = side == SIDE_OUT ? (div ? OUT_DIV_NTAP : OUT_MUL_TAP) : OUT_NONE;
        a.tg_op = tg ? TG_OUT : TG_NONE;
        float *tg_rows = tg ? (shared ? part : taps_bar) : nullptr;
        hipError_t e = plain_run(a, reinterpret_cast<const c32 *>(in), ws0, ws1, tg_rows, s);
        if (e == hipSuccess && tg && shared)
            e = rows_reduce(part, nblocks, N, part + nblocks * N, taps_bar, s);
        if (e != hipSuccess) {
            set_error("plain launch", e);
            return TF_EHIP;
        }
        return TF_OK;
    }

    Geometry g{};
    const c32 *tw = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        rc = fused_geometry(dev, K, M, nblocks, side, tg, tg && shared, &g, &tw, ws_caps_grid ? ws_bytes : 0);
    }
    if (rc) return rc;
    float *part = nullptr;
    if (tg && shared) {
        const size_t need = fused_ws_bytes(g.rows, N);
        if (!ws || ws_bytes < need || !aligned(ws, 4)) return TF_EWORKSPACE;
        part = reinterpret_cast<float *>(ws);
    }
    const FusedEntry &e = registry().entries[g.idx];
    FusedArgs a{};
    a.in = reinterpret_cast<const c32 *>(in);
    a.out = reinterpret_cast<c32 *>(out);
    a.taps = taps;
    a.aux = reinterpret_cast<const c32 *>(aux);
    a.tapbar = tg ? (shared ? part : taps_bar) : nullptr;
    a.status = status;
    a.tw = tw;
    a.nblocks = nblocks;
    a.tap_stride = tap_stride;
    a.div = div;
    hipError_t he = e.launch[side][tg ? 1 : 0](a, g.grid, s);
    if (he == hipSuccess && tg && shared)
        he = rows_reduce(part, g.rows, N, part + g.rows * N, taps_bar, s);
    if (he != hipSuccess) {
        set_error("fused launch", he);
        return TF_EHIP;
    }
    return TF_OK;
}

extern "C" int transform_forward(const void *coeffs, const float *taps, void *samples, int64_t nblocks,
                                 int32_t K, int32_t M, int64_t tap_stride, int32_t compute,
                                 void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = check_common(coeffs, taps, samples, nblocks, K, M, tap_stride, compute);
    if (rc || nblocks == 0) return rc;
    if (compute == TF_SPLIT_BF16 || compute == TF_SPLIT_FP16)
        return split_run(0, coeffs, taps, samples, nblocks, K, M, tap_stride, compute, workspace,
                         workspace_bytes, stream);
    return run(coeffs, taps, samples, nullptr, nullptr, nullptr, nblocks, K, M, tap_stride, compute,
               SIDE_IN, 0, false, workspace, workspace_bytes, stream);
}

extern "C" int transform_inverse(const void *samples, const float *taps, void *coeffs, int64_t nblocks,
                                 int32_t K, int32_t M, int64_t tap_stride, int32_t compute,
                                 int32_t *status_dev, void *workspace, size_t workspace_bytes,
                                 void *stream)
{
    int rc = check_common(samples, taps, coeffs, nblocks, K, M, tap_stride, compute);
    if (rc || nblocks == 0) return rc;
    if (status_dev && !aligned(status_dev, 4)) return TF_EINVAL;
    if (compute == TF_SPLIT_BF16 || compute == TF_SPLIT_FP16) return TF_EUNSUPPORTED;
    return run(samples, taps, coeffs, nullptr, nullptr, status_dev, nblocks, K, M, tap_stride,
               compute, SIDE_OUT, 1, false, workspace, workspace_bytes, stream);
}

extern "C" int transform_adjoint(const void *samples_bar, const float *taps, const void *coeffs,
                                 void *coeffs_bar, float *taps_bar, int64_t nblocks, int32_t K,
                                 int32_t M, int64_t tap_stride, int32_t compute, void *workspace,
                                 size_t workspace_bytes, void *stream)
{
    int rc = check_common(samples_bar, taps, coeffs_bar, nblocks, K, M, tap_stride, compute);
    if (rc || nblocks == 0) return rc;
    const int64_t N = int64_t(K) * M;
    if (taps_bar) {
        if (!coeffs || !aligned(coeffs, 8) || !aligned(taps_bar, 4)) return TF_EINVAL;
        if (overlap(coeffs, coeffs_bar, size_t(nblocks) * N * 8)) return TF_EINVAL;
        const size_t tb_bytes = size_t(tap_stride == 0 ? 1 : nblocks) * N * 4;
        const size_t x_bytes = size_t(nblocks) * N * 8;
        if (overlap2(taps_bar, tb_bytes, coeffs_bar, x_bytes) ||
            overlap2(taps_bar, tb_bytes, samples_bar, x_bytes) ||
            overlap2(taps_bar, tb_bytes, coeffs, x_bytes))
            return TF_EINVAL;
    }
    if (compute == TF_SPLIT_BF16 || compute == TF_SPLIT_FP16) {
        if (taps_bar) return TF_EUNSUPPORTED;
        return split_run(1, samples_bar, taps, coeffs_bar, nblocks, K, M, tap_stride, compute,
                         workspace, workspace_bytes, stream);
    }
    return run(samples_bar, taps, coeffs_bar, coeffs, taps_bar, nullptr, nblocks, K, M, tap_stride,
               compute, SIDE_OUT, 0, taps_bar != nullptr, workspace, workspace_bytes, stream);
}

// ------------------------------------------------------------------ allocation-free adjoint
// Scratch of transform_adjoint_noalloc: the shared tap gradient's partial rows and chunk
// sums.  One copy per GPU, held until the process ends.  Host code never uses the name
// itself as an address: each device's address comes from hipGetSymbolAddress.
constexpr size_t kNoallocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) float scratch[kNoallocScratchBytes / sizeof(float)];

// this device's address of `scratch`, looked up once per device with the device current
// (called under g_mu)
static int noalloc_scratch(int dev, float **ptr)
{
    DeviceState &d = dev_state(dev);
    if (!d.scratch) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch)", e);
            return TF_EHIP;
        }
        d.scratch = static_cast<float *>(p);
    }
    *ptr = d.scratch;
    return TF_OK;
}

extern "C" size_t transform_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

extern "C" int transform_adjoint_noalloc(const void *samples_bar, const float *taps, const void *coeffs,
                                         void *coeffs_bar, float *taps_bar, int64_t nblocks, int32_t K,
                                         int32_t M, int64_t tap_stride, void *stream)
{
    int rc = check_common(samples_bar, taps, coeffs_bar, nblocks, K, M, tap_stride, TF_FP32);
    if (rc || nblocks == 0) return rc;
    const int64_t N = int64_t(K) * M;
    if (taps_bar) {
        if (!coeffs || !aligned(coeffs, 8) || !aligned(taps_bar, 4)) return TF_EINVAL;
        if (overlap(coeffs, coeffs_bar, size_t(nblocks) * N * 8)) return TF_EINVAL;
        const size_t tb_bytes = size_t(tap_stride == 0 ? 1 : nblocks) * N * 4;
        const size_t x_bytes = size_t(nblocks) * N * 8;
        if (overlap2(taps_bar, tb_bytes, coeffs_bar, x_bytes) ||
            overlap2(taps_bar, tb_bytes, samples_bar, x_bytes) ||
            overlap2(taps_bar, tb_bytes, coeffs, x_bytes))
            return TF_EINVAL;
    }
    float *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        int dev = 0;
        rc = current_device(&dev);
        if (!rc) rc = noalloc_scratch(dev, &ws);
    }
    if (rc) return rc;
    // the shared tap gradient's partial rows go to the scratch array, the grid capped so that
    // they fit; every row is written in full by the kernel, so nothing needs clearing
    return run(samples_bar, taps, coeffs_bar, coeffs, taps_bar, nullptr, nblocks, K, M, tap_stride,
               TF_FP32, SIDE_OUT, 0, taps_bar != nullptr, ws, kNoallocScratchBytes, stream, true);
}

extern "C" int transform_inverse_adjoint(const void *coeffs_bar, const float *taps, const void *coeffs,
                                         void *samples_bar, float *taps_bar, int64_t nblocks,
                                         int32_t K, int32_t M, int64_t tap_stride, int32_t compute,
                                         void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = check_common(coeffs_bar, taps, samples_bar, nblocks, K, M, tap_stride, compute);
    if (rc || nblocks == 0) return rc;
    if (compute != TF_FP32) return TF_EUNSUPPORTED;
    const int64_t N = int64_t(K) * M;
    if (taps_bar) {
        if (!coeffs || !aligned(coeffs, 8) || !aligned(taps_bar, 4)) return TF_EINVAL;
        if (overlap(coeffs, samples_bar, size_t(nblocks) * N * 8)) return TF_EINVAL;
    }
    return run(coeffs_bar, taps, samples_bar, coeffs, taps_bar, nullptr, nblocks, K, M, tap_stride,
               compute, SIDE_IN, 1, taps_bar != nullptr, workspace, workspace_bytes, stream);
}

extern "C" int transform_prepare(int32_t K, int32_t M, int32_t compute)
{
    if (!supported_km(K, M)) return TF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    if (compute == TF_PLAIN_FP32) {
        const c32 *r = nullptr;
        return plain_roots(dev, K, M, &r);
    }
    if (compute == TF_SPLIT_BF16 || compute == TF_SPLIT_FP16) return split_prepare(K, M, compute);
    int cap = 0;
    int idx = chosen_entry(K, M, &cap);
    if (idx < 0) return TF_EUNSUPPORTED;
    const c32 *tw = nullptr;
    int occ = 0;
    return entry_tables(dev, idx, SIDE_IN, false, &tw, &occ);
}

extern "C" const char *transform_status_string(int status)
{
    switch (status) {
    case TF_OK: return "TF_OK";
    case TF_EINVAL: return "TF_EINVAL: invalid argument";
    case TF_EUNSUPPORTED: return "TF_EUNSUPPORTED: unsupported size or compute mode";
    case TF_ESINGULAR: return "TF_ESINGULAR: singular filter";
    case TF_EHIP: return "TF_EHIP: HIP runtime error";
    case TF_EWORKSPACE: return "TF_EWORKSPACE: workspace missing or too small";
    default: return "unknown status";
    }
}

extern "C" const char *transform_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ schedules
extern "C" int transform_schedule_count(int32_t K, int32_t M)
{
    if (!supported_km(K, M)) return 0;
    auto &r = registry();
    auto it = r.by_km.find({K, M});
    return it == r.by_km.end() ? 0 : (int)it->second.size();
}

extern "C" int transform_schedule_describe(int32_t K, int32_t M, int32_t idx, char *buf, size_t buflen)
{
    if (!supported_km(K, M) || !buf) return TF_EINVAL;
    auto &r = registry();
    auto it = r.by_km.find({K, M});
    if (it == r.by_km.end() || idx < 0 || idx >= (int)it->second.size()) return TF_EINVAL;
    const FusedEntry &e = r.entries[it->second[idx]];
    std::string rad;
    for (int i = 0; i < e.npass; ++i) rad += (i ? "," : "") + std::to_string(e.radix[i]);
    std::snprintf(buf, buflen,
                  "{\"K\": %d, \"M\": %d, \"radices\": [%s], \"threads_per_block\": %d, "
                  "\"blocks_per_workgroup\": %d, \"lds_bytes\": %d, \"prefetch\": %s, "
                  "\"sequential_twiddles\": %s, \"paired_io\": %s, \"nontemporal\": %s, \"early_fetch\": %s, "
                  "\"half_lds\": %s}",
                  e.K, e.M, rad.c_str(), e.TB, e.BPW, e.lds_bytes, (e.opt & OPT_NO_PREFETCH) ? "false" : "true",
                  (e.opt & OPT_SEQ_TWIDDLE) ? "true" : "false", (e.opt & OPT_PAIRED_IO) ? "true" : "false",
                  (e.opt & OPT_NT) ? "true" : "false", (e.opt & OPT_EARLY_FETCH) ? "true" : "false",
                  (e.opt & OPT_HALF_LDS) ? "true" : "false");
    return TF_OK;
}

extern "C" int transform_schedule_selected(int32_t K, int32_t M, int32_t *idx, int32_t *grid_cap)
{
    if (!supported_km(K, M) || !idx || !grid_cap) return TF_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    *idx = 0;
    *grid_cap = 0;
    auto s = g_select.find({K, M});
    if (s != g_select.end()) {
        *idx = s->second.idx < 0 ? 0 : s->second.idx;
        *grid_cap = s->second.grid_cap;
    }
    return TF_OK;
}

extern "C" int transform_schedule_select(int32_t K, int32_t M, int32_t idx, int32_t grid_cap)
{
    if (!supported_km(K, M)) return TF_EUNSUPPORTED;
    if (idx >= transform_schedule_count(K, M) || grid_cap < 0) return TF_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Selection s;
    s.idx = idx;
    s.grid_cap = grid_cap;
    g_select[{K, M}] = s;
    return TF_OK;
}

extern "C" int transform_save_schedule(const char *path)
{
    if (!path) return TF_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    FILE *f = std::fopen(path, "w");
    if (!f) return TF_EINVAL;
    std::fprintf(f, "{");
    bool first = true;
    for (auto &kv : g_select) {
        std::fprintf(f, "%s\n  \"%d,%d\": [%d, %d]", first ? "" : ",", kv.first.first, kv.first.second,
                     kv.second.idx, kv.second.grid_cap);
        first = false;
    }
    std::fprintf(f, "\n}\n");
    std::fclose(f);
    return TF_OK;
}

extern "C" int transform_load_schedule(const char *path)
{
    if (!path) return TF_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return TF_EINVAL;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
    // entries look like  "K,M": [idx, cap]
    size_t pos = 0;
    int loaded = 0;
    while ((pos = txt.find('"', pos)) != std::string::npos) {
        int K = 0, M = 0, idx = 0, cap = 0;
        if (std::sscanf(txt.c_str() + pos, "\"%d,%d\" : [ %d , %d ]", &K, &M, &idx, &cap) == 4 ||
            std::sscanf(txt.c_str() + pos, "\"%d,%d\": [%d, %d]", &K, &M, &idx, &cap) == 4) {
            if (transform_schedule_select(K, M, idx, cap) != TF_OK) return TF_EINVAL;
            ++loaded;
        }
        size_t close = txt.find('"', pos + 1);
        if (close == std::string::npos) break;
        pos = close + 1;
    }
    return loaded >= 0 ? TF_OK : TF_EINVAL;
}
