// Fused block-transform kernel for gfx950: one workgroup owns BPW blocks of
// N = K*M points and runs every stage of the transform on them between one
// coalesced HBM read and one coalesced HBM write.
//
// The forward evaluates y_u = sum_n Lambda_n S_n exp(+j 2 pi n u / N) -- the
// filtered trigonometric polynomial of eq. (6) on the uniform grid, whose
// u = M q coset is eq. (7).  It is computed as a self-sorting (Stockham) FFT
// whose first radix is M: that pass is the circular fold of eq. (7) (length-M
// DFT over n = p + K r, applied to the filtered coefficients), and the
// remaining power-of-two radices form the length-K IDFT with its coset
// twiddles.  Natural order in, natural order out.
//
// Pass p (radix R, stride Ns = product of earlier radices) on butterfly j:
//   v_r = x[j + r N/R],  v_r *= exp(+j 2 pi (j mod Ns) r / (Ns R)),  v = DFT_R(v),
//   x'[(j / Ns) Ns R + (j mod Ns) + r Ns] = v_r.
// Pass 0 reads HBM (and applies the input-side filter), the last pass writes
// HBM (and applies the output-side filter); the passes in between run
// in place in LDS, each thread holding its butterflies in registers across
// the barrier.
//
// The negative-exponent transforms (inverse of eq. (31), the adjoint) run the
// same code with inputs and outputs conjugated.
#pragma once

#include "bt_dft.hpp"

namespace bt {

enum InOp : int { IN_NONE = 0, IN_MUL_TAP = 1, IN_DIV_NTAP = 2 };
enum OutOp : int { OUT_NONE = 0, OUT_MUL_TAP = 1, OUT_DIV_NTAP = 2 };
enum TgOp : int {
    TG_NONE = 0,
    TG_OUT = 1,   // Re(conj(aux_n) W_n), W taken before the output filter (forward's adjoint)
    TG_IN = 2,    // -Re(conj(g_n) aux_n) / Lambda_n at the input (inverse's adjoint)
};

struct FusedArgs {
    const c32 *in;
    c32 *out;
    const float *taps;
    const c32 *aux;       // S (TG_OUT) or the inverse's output (TG_IN)
    float *tapbar;        // per block [B][N] when tap_stride != 0, else partial rows [grid*BPW][N]
    int *status;          // set to 1 when a zero tap is met by IN/OUT_DIV_NTAP (nullable)
    const c32 *tw;        // per-pass twiddle table of the plan
    int64_t nblocks;
    int64_t tap_stride;   // 0: one tap vector for all blocks; N: one per block
    int conj_io;
    int in_op, out_op, tg_op;
};

template <int... Rs>
struct Radices {
    static constexpr int count = sizeof...(Rs);
    static constexpr int get(int i)
    {
        constexpr int a[] = {Rs...};
        return a[i];
    }
    static constexpr int total()
    {
        int p = 1;
        for (int q = 0; q < count; ++q) p *= get(q);
        return p;
    }
    static constexpr int ns(int i)
    {
        int p = 1;
        for (int q = 0; q < i; ++q) p *= get(q);
        return p;
    }
    // twiddle-table offset of pass i (passes >= 1 own Ns*R entries each)
    static constexpr int tw_off(int i)
    {
        int o = 0;
        for (int q = 1; q < i; ++q) o += ns(q) * get(q);
        return o;
    }
    static constexpr int tw_total() { return tw_off(count); }
    static constexpr int max_nb()
    {
        int m = 0;
        for (int q = 0; q < count; ++q) m = (total() / get(q) > m) ? total() / get(q) : m;
        return m;
    }
};

template <int M, class KR>
struct PrependM;
template <int M, int... Rs>
struct PrependM<M, Radices<Rs...>> {
    using type = Radices<M, Rs...>;
};
template <int... Rs>
struct PrependM<1, Radices<Rs...>> {
    using type = Radices<Rs...>;
};
template <>
struct PrependM<1, Radices<>> {
    using type = Radices<1>;
};

// ------------------------------------------------------------------ element ops
BT_HD c32 load_c(const c32 *p) { return *p; }

__device__ __forceinline__ c32 in_transform(const FusedArgs &a, c32 x, const float *tp, int64_t n,
                                             float Nf, const c32 *auxb, float *tg)
{
    if (a.in_op == IN_DIV_NTAP && a.tg_op == TG_IN) {
        // -Re(conj(g_n) Shat_n) / Lambda_n, from the unconjugated input
        *tg = -(x.x * auxb[n].x + x.y * auxb[n].y) / tp[n];
    }
    if (a.conj_io) x = conj(x);
    if (a.in_op == IN_MUL_TAP) {
        x = scale(x, tp[n]);
    } else if (a.in_op == IN_DIV_NTAP) {
        const float t = tp[n];
        if (t == 0.0f && a.status) *a.status = 1;
        x = scale(x, 1.0f / (Nf * t));
    }
    return x;
}

__device__ __forceinline__ c32 out_transform(const FusedArgs &a, c32 w, const float *tp, int64_t k,
                                              float Nf, const c32 *auxb, float *tg)
{
    if (a.conj_io) w = conj(w);
    if (a.tg_op == TG_OUT) *tg = auxb[k].x * w.x + auxb[k].y * w.y;
    if (a.out_op == OUT_MUL_TAP) {
        w = scale(w, tp[k]);
    } else if (a.out_op == OUT_DIV_NTAP) {
        const float t = tp[k];
        if (t == 0.0f && a.status) *a.status = 1;
        w = scale(w, 1.0f / (Nf * t));
    }
    return w;
}

// ------------------------------------------------------------------ passes
template <class PL, int TB, int P>
__device__ __forceinline__ void lds_passes(c32 *L, int tid, const c32 *tw)
{
    if constexpr (P < PL::count - 1) {
        constexpr int N = PL::total();
        constexpr int R = PL::get(P);
        constexpr int NS = PL::ns(P);
        constexpr int NB = N / R;
        constexpr int IT = (NB + TB - 1) / TB;
        constexpr int TWO = PL::tw_off(P);
        c32 v[IT][R];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = tid + i * TB;
            if (IT * TB == NB || j < NB) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[i][r] = L[j + r * NB];
                const int jm = j % NS;
                const c32 *t = tw + TWO + jm * R;
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], t[r]);
                dft<R>(v[i]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = tid + i * TB;
            if (IT * TB == NB || j < NB) {
                const int jm = j % NS;
                const int base = (j / NS) * NS * R + jm;
#pragma unroll
                for (int r = 0; r < R; ++r) L[base + r * NS] = v[i][r];
            }
        }
        __syncthreads();
        lds_passes<PL, TB, P + 1>(L, tid, tw);
    }
}

template <class PL, int TB, int BPW>
__global__ void __launch_bounds__(TB *BPW) fused_kernel(FusedArgs a)
{
    constexpr int N = PL::total();
    constexpr int NP = PL::count;
    constexpr int R0 = PL::get(0);
    constexpr int NB0 = N / R0;
    constexpr int IT0 = (NB0 + TB - 1) / TB;
    constexpr int RL = PL::get(NP - 1);
    constexpr int NSL = PL::ns(NP - 1);
    constexpr int NBL = N / RL;
    constexpr int ITL = (NBL + TB - 1) / TB;
    constexpr int TWL = PL::tw_off(NP - 1);
    // tap-gradient accumulators live on the side of the pass that computes them
    constexpr int TGI = (IT0 * R0 > ITL * RL) ? IT0 * R0 : ITL * RL;

    __shared__ c32 lds[NP > 1 ? BPW * N : 1];
    const int bi = threadIdx.x / TB;
    const int tid = threadIdx.x - bi * TB;
    c32 *L = lds + (NP > 1 ? bi * N : 0);
    const float Nf = float(N);
    const bool shared_taps = (a.tap_stride == 0);

    float acc[TGI];
#pragma unroll
    for (int q = 0; q < TGI; ++q) acc[q] = 0.0f;

    for (int64_t g = blockIdx.x; g * BPW < a.nblocks; g += gridDim.x) {
        const int64_t blk = g * BPW + bi;
        const bool valid = blk < a.nblocks;
        const c32 *inb = a.in + blk * N;
        c32 *outb = a.out + blk * N;
        const float *tp = a.taps + blk * a.tap_stride;
        const c32 *auxb = a.aux ? a.aux + blk * N : nullptr;
        float *tgb = a.tapbar + (shared_taps ? 0 : blk * N);

        if constexpr (NP == 1) {
            // the whole transform is one radix-N butterfly per block
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (valid && (IT0 * TB == NB0 || j < NB0)) {
                    c32 v[R0];
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        float tg = 0.f;
                        v[r] = in_transform(a, inb[j + r * NB0], tp, j + r * NB0, Nf, auxb, &tg);
                        if (a.tg_op == TG_IN) {
                            if (shared_taps) acc[i * R0 + r] += tg;
                            else tgb[j + r * NB0] = tg;
                        }
                    }
                    dft<R0>(v);
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        const int k = j + r * NB0;
                        float tg = 0.f;
                        outb[k] = out_transform(a, v[r], tp, k, Nf, auxb, &tg);
                        if (a.tg_op == TG_OUT) {
                            if (shared_taps) acc[i * R0 + r] += tg;
                            else tgb[k] = tg;
                        }
                    }
                }
            }
        } else {
            // ---- pass 0: HBM -> registers -> DFT_R0 -> LDS (no twiddle, Ns = 1)
            c32 v0[IT0][R0];
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (valid && (IT0 * TB == NB0 || j < NB0)) {
#pragma unroll
                    for (int r = 0; r < R0; ++r) {
                        float tg = 0.f;
                        v0[i][r] = in_transform(a, inb[j + r * NB0], tp, j + r * NB0, Nf, auxb, &tg);
                        if (a.tg_op == TG_IN) {
                            if (shared_taps) acc[i * R0 + r] += tg;
                            else tgb[j + r * NB0] = tg;
                        }
                    }
                    dft<R0>(v0[i]);
                }
            }
            __syncthreads();   // the previous group's last pass has finished reading LDS
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (valid && (IT0 * TB == NB0 || j < NB0)) {
#pragma unroll
                    for (int r = 0; r < R0; ++r) L[j * R0 + r] = v0[i][r];
                }
            }
            __syncthreads();

            // ---- middle passes in LDS
            lds_passes<PL, TB, 1>(L, tid, a.tw);

            // ---- last pass: LDS -> registers -> twiddle -> DFT_RL -> HBM
#pragma unroll
            for (int i = 0; i < ITL; ++i) {
                const int j = tid + i * TB;
                if (valid && (ITL * TB == NBL || j < NBL)) {
                    c32 v[RL];
#pragma unroll
                    for (int r = 0; r < RL; ++r) v[r] = L[j + r * NBL];
                    const c32 *t = a.tw + TWL + j * RL;    // j < NBL = NSL, so j mod NSL = j
#pragma unroll
                    for (int r = 1; r < RL; ++r) v[r] = cmul(v[r], t[r]);
                    dft<RL>(v);
#pragma unroll
                    for (int r = 0; r < RL; ++r) {
                        const int k = j + r * NSL;
                        float tg = 0.f;
                        outb[k] = out_transform(a, v[r], tp, k, Nf, auxb, &tg);
                        if (a.tg_op == TG_OUT) {
                            if (shared_taps) acc[i * RL + r] += tg;
                            else tgb[k] = tg;
                        }
                    }
                }
            }
        }
    }

    // ---- shared taps: one partial row of the tap gradient per (workgroup, block slot)
    if (a.tg_op != TG_NONE && shared_taps) {
        float *row = a.tapbar + (int64_t(blockIdx.x) * BPW + bi) * N;
        if (a.tg_op == TG_IN || NP == 1) {
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (IT0 * TB == NB0 || j < NB0) {
#pragma unroll
                    for (int r = 0; r < R0; ++r) row[j + r * NB0] = acc[i * R0 + r];
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITL; ++i) {
                const int j = tid + i * TB;
                if (ITL * TB == NBL || j < NBL) {
#pragma unroll
                    for (int r = 0; r < RL; ++r) row[j + r * NSL] = acc[i * RL + r];
                }
            }
        }
    }
}

// sum of `rows` partial rows of length n: out[k] = sum_r part[r*n + k] (fixed order)
__global__ void tapgrad_reduce_kernel(const float *part, int64_t rows, int64_t n, float *out);

// ------------------------------------------------------------------ registry entry
typedef hipError_t (*fused_launch_fn)(const FusedArgs &, unsigned grid, hipStream_t);

struct FusedEntry {
    int K, M, TB, BPW, npass;
    int radix[8];
    int tw_entries;
    int lds_bytes;
    fused_launch_fn launch;
    const void *kernel;   // for occupancy queries
};

template <class PL, int TB, int BPW>
hipError_t fused_launch(const FusedArgs &a, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL((fused_kernel<PL, TB, BPW>), dim3(grid), dim3(TB * BPW), 0, s, a);
    return hipGetLastError();
}

template <class PL, int TB, int BPW>
FusedEntry make_entry(int K, int M)
{
    FusedEntry e{};
    e.K = K;
    e.M = M;
    e.TB = TB;
    e.BPW = BPW;
    e.npass = PL::count;
    for (int i = 0; i < PL::count && i < 8; ++i) e.radix[i] = PL::get(i);
    e.tw_entries = PL::tw_total();
    e.lds_bytes = PL::count > 1 ? BPW * PL::total() * (int)sizeof(c32) : 0;
    e.launch = &fused_launch<PL, TB, BPW>;
    e.kernel = reinterpret_cast<const void *>(&fused_kernel<PL, TB, BPW>);
    return e;
}

// default radix plan of the length-K part
template <int K> struct KPlan;
template <> struct KPlan<1> { using type = Radices<>; };
template <> struct KPlan<2> { using type = Radices<2>; };
template <> struct KPlan<4> { using type = Radices<4>; };
template <> struct KPlan<8> { using type = Radices<8>; };
template <> struct KPlan<16> { using type = Radices<16>; };
template <> struct KPlan<32> { using type = Radices<32>; };
template <> struct KPlan<64> { using type = Radices<8, 8>; };
template <> struct KPlan<128> { using type = Radices<16, 8>; };
template <> struct KPlan<256> { using type = Radices<16, 16>; };
template <> struct KPlan<512> { using type = Radices<16, 32>; };
template <> struct KPlan<1024> { using type = Radices<32, 32>; };

constexpr int pow2_floor(int x)
{
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

template <class PL>
struct DefaultShape {
    static constexpr int TB0 = pow2_floor(PL::max_nb());
    static constexpr int TB = TB0 > 512 ? 512 : TB0;
    static constexpr int BPW0 = TB >= 256 ? 1 : 256 / TB;
    // keep a workgroup's LDS within 64 KB so several groups share a CU
    static constexpr int lds1 = PL::total() * 8;
    static constexpr int BPW = (BPW0 * lds1 > 65536 && BPW0 > 1) ? (65536 / lds1 > 0 ? pow2_floor(65536 / lds1) : 1) : BPW0;
};

template <int K, int M>
FusedEntry default_entry()
{
    using PL = typename PrependM<M, typename KPlan<K>::type>::type;
    using SH = DefaultShape<PL>;
    return make_entry<PL, SH::TB, SH::BPW>(K, M);
}

} // namespace bt
