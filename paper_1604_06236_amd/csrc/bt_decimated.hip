// Decimated operator of eq. (7) and its adjoint.
//
// eq. (7) evaluates the polynomial of eq. (6), with R = eta P coefficients, at
// the P regular points q/P only: a filter multiply, a circular fold of the
// length-R spectrum onto P bins and a length-P IDFT.  With P = K, eta = M,
// N = K M, per block:
//   forward  out_q  = sum_{n<N} Lambda_n S_n e^{+j 2 pi n q / K}
//                   = sum_{p<K} (sum_{r<M} Lambda_{p+Kr} S_{p+Kr}) e^{+j 2 pi p q / K},   q < K
//   adjoint  Sbar_n = Lambda_n sum_{q<K} ybar_q e^{-j 2 pi n q / K}                     n < N
// (with the log-series filter of eq. (41) and a delta train on a uniform fine
// grid this is the v(q/P) step of eq. (28)).
//
// The K-point transform is a Stockham FFT in LDS (same pass machinery as the
// full operator).  Forward: all threads fold the M cosets into natural-order
// LDS, the passes run in LDS and the last one writes the K outputs.  Adjoint:
// conjugated input into LDS, every pass in LDS, then all threads write each of
// the K results to its M cosets, times the filter ("unfold").  M is a runtime
// parameter.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <vector>

#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"
#include "bt_fused.hpp"

namespace bt {

struct DecArgs {
    const c32 *in;
    c32 *out;
    const float *taps;
    const c32 *tw;
    int64_t nblocks;
    int64_t tap_stride;   // 0 or N
    int M;
};

template <class PL, int TB, int SIDE>
__global__ void __launch_bounds__(TB) decimated_kernel(DecArgs a)
{
    constexpr int K = PL::total();
    constexpr int NP = PL::count;
    constexpr int RL = PL::get(NP - 1);
    constexpr int NSL = PL::ns(NP - 1);
    constexpr int NBL = K / RL;
    constexpr int ITL = (NBL + TB - 1) / TB;
    constexpr int OPT = OPT_SEQ_TWIDDLE;
    constexpr uint32_t CB = 8, FB = 4;
    static_assert(NP >= 2, "K must take at least two radix passes");
    __shared__ c32 L[K];
    poison_lds(L, K);

    const int tid = threadIdx.x;
    const int M = a.M;
    const int64_t N = int64_t(K) * M;
    const bool shared_taps = a.tap_stride == 0;

    c32 w1s[TwSlots<PL, TB, OPT>::total()];
    static_for<1, NP>([&](auto pI) {
        constexpr int P = decltype(pI)::value;
        constexpr int NB = K / PL::get(P);
        constexpr int IT = TwSlots<PL, TB, OPT>::it(P);
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = tid + i * TB;
            w1s[TwSlots<PL, TB, OPT>::off(P) + i] = (j < NB) ? a.tw[PL::tw_off(P) + j % PL::ns(P)] : c32{1.f, 0.f};
        }
    });

    constexpr int ITK = (K + TB - 1) / TB;     // natural-order points per thread
    for (int64_t b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
        const uint32_t in_len = SIDE == SIDE_IN ? uint32_t(N) : uint32_t(K);
        const uint32_t out_len = SIDE == SIDE_IN ? uint32_t(K) : uint32_t(N);
        const rsrc_t ri = make_rsrc(a.in + b * in_len, in_len * CB);
        const rsrc_t ro = make_rsrc(a.out + b * out_len, out_len * CB);
        const rsrc_t rt = make_rsrc(a.taps + (shared_taps ? 0 : b * N), uint32_t(N) * FB);

        // ---- into LDS in natural order: the fold sum_r Lambda S at p + r K (forward),
        //      or the conjugated input (adjoint); all threads, coalesced
        c32 u[ITK];
        if constexpr (SIDE == SIDE_IN) {
#pragma unroll
            for (int i = 0; i < ITK; ++i) u[i] = c32{0.f, 0.f};
            for (int r = 0; r < M; ++r) {
                c32 s[ITK];
                float t[ITK];
#pragma unroll
                for (int i = 0; i < ITK; ++i) {
                    const uint32_t n = uint32_t(tid + i * TB + r * K);
                    s[i] = ld_c(ri, n * CB, 0);
                    t[i] = ld_f(rt, n * FB, 0);
                }
#pragma unroll
                for (int i = 0; i < ITK; ++i) {
                    u[i].x += t[i] * s[i].x;
                    u[i].y += t[i] * s[i].y;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITK; ++i) u[i] = conj(ld_c(ri, uint32_t(tid + i * TB) * CB, 0));
        }
        lds_barrier();   // the previous block has finished reading LDS
#pragma unroll
        for (int i = 0; i < ITK; ++i)
            if (ITK * TB == K || tid + i * TB < K) L[tid + i * TB] = u[i];
        lds_barrier();

        if constexpr (SIDE == SIDE_IN) {
            // ---- every pass but the last in LDS, the last one writes the K outputs
            lds_passes<PL, TB, 0, OPT>(L, tid, w1s);
            constexpr int SLOTL = TwSlots<PL, TB, OPT>::off(NP - 1);
#pragma unroll
            for (int i = 0; i < ITL; ++i) {
                const int j = tid + i * TB;
                if (j < NBL) {
                    c32 v[RL];
                    static_for<0, RL>([&](auto rI) {
                        constexpr int q = decltype(rI)::value;
                        v[q] = L[j + q * NBL];
                    });
                    twiddle<OPT, RL>(v, w1s[SLOTL + i]);
                    dft<RL>(v);
                    static_for<0, RL>([&](auto rI) {
                        constexpr int q = decltype(rI)::value;
                        st_c(v[q], ro, uint32_t(j + q * NSL) * CB, 0);
                    });
                }
            }
        } else {
            // ---- all passes in LDS (natural-order result), then the unfold: W_p to
            //      every coset p + r K, times the filter; all threads, coalesced
            lds_passes<PL, TB, 0, OPT, NP>(L, tid, w1s);
#pragma unroll
            for (int i = 0; i < ITK; ++i)
                if (ITK * TB == K || tid + i * TB < K) u[i] = conj(L[tid + i * TB]);
            // non-temporal stores: the N outputs are not read again soon, and keeping them out
            // of the caches leaves less to write back under the next launch's reads
            for (int r = 0; r < M; ++r) {
                float t[ITK];
#pragma unroll
                for (int i = 0; i < ITK; ++i) t[i] = ld_f(rt, uint32_t(tid + i * TB + r * K) * FB, 0);
#pragma unroll
                for (int i = 0; i < ITK; ++i)
                    if (ITK * TB == K || tid + i * TB < K)
                        st_c<2>(scale(u[i], t[i]), ro, uint32_t(tid + i * TB + r * K) * CB, 0);
            }
        }
    }
}

// ------------------------------------------------------------------ host side
typedef hipError_t (*dec_launch_fn)(const DecArgs &, unsigned, hipStream_t);

template <class PL, int TB, int SIDE>
static hipError_t dec_launch(const DecArgs &a, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL((decimated_kernel<PL, TB, SIDE>), dim3(grid), dim3(TB), 0, s, a);
    return hipGetLastError();
}

struct DecEntry {
    int K, TB, npass;
    int radix[8];
    dec_launch_fn launch[2];
};

template <class PL, int TB>
static DecEntry dec_entry()
{
    DecEntry e{};
    e.K = PL::total();
    e.TB = TB;
    e.npass = PL::count;
    for (int i = 0; i < PL::count; ++i) e.radix[i] = PL::get(i);
    e.launch[0] = &dec_launch<PL, TB, SIDE_IN>;
    e.launch[1] = &dec_launch<PL, TB, SIDE_OUT>;
    return e;
}

static const DecEntry *dec_find(int K)
{
    static const DecEntry table[] = {
        dec_entry<Radices<4, 4>, 16>(),      dec_entry<Radices<4, 8>, 32>(),
        dec_entry<Radices<8, 8>, 64>(),      dec_entry<Radices<16, 8>, 128>(),
        dec_entry<Radices<16, 16>, 256>(),   dec_entry<Radices<8, 8, 8>, 512>(),
        dec_entry<Radices<16, 16, 4>, 1024>(),
    };
    for (const DecEntry &e : table)
        if (e.K == K) return &e;
    return nullptr;
}

static std::mutex g_dec_mu;
static std::map<std::pair<int, int>, c32 *> g_dec_tw;   // (device, K) -> base roots

static int dec_twiddles(const DecEntry &e, const c32 **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TF_EHIP;
    std::lock_guard<std::mutex> lk(g_dec_mu);
    auto it = g_dec_tw.find({dev, e.K});
    if (it == g_dec_tw.end()) {
        std::vector<c32> h;
        long ns = e.radix[0];
        for (int p = 1; p < e.npass; ++p) {
            const long R = e.radix[p];
            for (long jm = 0; jm < ns; ++jm) {
                const double ang = 2.0 * M_PI * double(jm) / double(ns * R);
                h.push_back(c32{float(std::cos(ang)), float(std::sin(ang))});
            }
            ns *= R;
        }
        c32 *d = nullptr;
        hipError_t er = hipMalloc(&d, h.size() * sizeof(c32));
        if (er == hipSuccess) er = hipMemcpy(d, h.data(), h.size() * sizeof(c32), hipMemcpyHostToDevice);
        if (er != hipSuccess) {
            set_error("decimated twiddles", er);
            return TF_EHIP;
        }
        it = g_dec_tw.emplace(std::make_pair(dev, e.K), d).first;
    }
    *out = it->second;
    return TF_OK;
}

static int dec_run(int side, const void *in, const float *taps, void *out, int64_t nblocks, int32_t K,
                   int32_t M, int64_t tap_stride, void *stream)
{
    const DecEntry *e = dec_find(K);
    if (!e || M < 1 || M > 4096) return TF_EUNSUPPORTED;
    const int64_t N = int64_t(K) * M;
    if (nblocks < 0 || (tap_stride != 0 && tap_stride != N)) return TF_EINVAL;
    if (N * 8 > 0x7fffffffLL) return TF_EUNSUPPORTED;
    if (nblocks == 0) return TF_OK;
    if (!in || !out || !taps) return TF_EINVAL;
    const uintptr_t pin = reinterpret_cast<uintptr_t>(in), pout = reinterpret_cast<uintptr_t>(out);
    if (pin % 8 || pout % 8 || reinterpret_cast<uintptr_t>(taps) % 4) return TF_EINVAL;
    const size_t in_bytes = size_t(nblocks) * (side == SIDE_IN ? N : K) * 8;
    const size_t out_bytes = size_t(nblocks) * (side == SIDE_IN ? K : N) * 8;
    if (pin < pout + out_bytes && pout < pin + in_bytes) return TF_EINVAL;
    const c32 *tw = nullptr;
    int rc = dec_twiddles(*e, &tw);
    if (rc) return rc;
    DecArgs a{};
    a.in = reinterpret_cast<const c32 *>(in);
    a.out = reinterpret_cast<c32 *>(out);
    a.taps = taps;
    a.tw = tw;
    a.nblocks = nblocks;
    a.tap_stride = tap_stride;
    a.M = M;
    const unsigned grid = unsigned(std::min<int64_t>(nblocks, 1 << 20));
    hipError_t er = e->launch[side](a, grid, reinterpret_cast<hipStream_t>(stream));
    if (er != hipSuccess) {
        set_error("decimated launch", er);
        return TF_EHIP;
    }
    return TF_OK;
}

} // namespace bt

using namespace bt;

extern "C" int transform_decimated(const void *coeffs, const float *taps, void *samples, int64_t nblocks,
                                   int32_t K, int32_t M, int64_t tap_stride, void *stream)
{
    return dec_run(SIDE_IN, coeffs, taps, samples, nblocks, K, M, tap_stride, stream);
}

extern "C" int transform_decimated_adjoint(const void *samples_bar, const float *taps, void *coeffs_bar,
                                           int64_t nblocks, int32_t K, int32_t M, int64_t tap_stride,
                                           void *stream)
{
    return dec_run(SIDE_OUT, samples_bar, taps, coeffs_bar, nblocks, K, M, tap_stride, stream);
}
