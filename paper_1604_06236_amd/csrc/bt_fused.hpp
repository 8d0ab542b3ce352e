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

// Where the filter is applied.  SIDE_IN: positive exponent, filter on the
// input (forward: multiply by Lambda; adjoint of the inverse: divide by
// N Lambda).  SIDE_OUT: negative exponent (inputs and outputs conjugated),
// filter on the output (adjoint: multiply; inverse: divide).
enum Side : int { SIDE_IN = 0, SIDE_OUT = 1 };

struct FusedArgs {
    const c32 *in;
    c32 *out;
    const float *taps;
    const c32 *aux;       // S (output-side tap term) or the inverse's output (input side)
    float *tapbar;        // per block [B][N] when tap_stride != 0, else partial rows [grid*BPW][N]
    int *status;          // set to 1 when a divide meets a zero tap (nullable)
    const c32 *tw;        // base twiddles of the plan
    int64_t nblocks;
    int64_t tap_stride;   // 0: one tap vector for all blocks; N: one per block
    int div;              // 0: multiply by Lambda_n; 1: divide by N Lambda_n
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
    // offset of pass i's base roots in the twiddle table (passes >= 1 own Ns entries each)
    static constexpr int tw_off(int i)
    {
        int o = 0;
        for (int q = 1; q < i; ++q) o += ns(q);
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

// ------------------------------------------------------------------ helpers
// Workgroup barrier that orders LDS only: global loads issued before it stay in
// flight (a full __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Test builds (BT_POISON_LDS defined) fill a kernel's LDS with NaN on entry, so that a
// read of an element that no thread has written in this launch (a missing store or a
// barrier in the wrong place) turns the affected outputs into NaN.  No-op otherwise.
__device__ __forceinline__ void poison_lds(c32 *p, int n)
{
#ifdef BT_POISON_LDS
    const float nan = __builtin_nanf("");
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = c32{nan, nan};
    __syncthreads();
#else
    (void)p;
    (void)n;
#endif
}

// v_r *= w1^r for r = 1..R-1; the powers come from one base root by squaring
// and single multiplications (at most 2 log2 R products deep)
template <int R>
__device__ __forceinline__ void apply_twiddles(c32 (&v)[R], c32 w1)
{
    if constexpr (R > 1) {
        c32 w[R];
        w[1] = w1;
        static_for<2, R>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            if constexpr (r % 2 == 0) {
                const c32 h = w[r / 2];
                w[r] = c32{h.x * h.x - h.y * h.y, 2.0f * h.x * h.y};
            } else {
                w[r] = cmul(w[r - 1], w1);
            }
        });
        static_for<1, R>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            v[r] = cmul(v[r], w[r]);
        });
    }
}

// the same with the powers formed one after another (two live registers, error
// growing with r instead of log2 r)
template <int R>
__device__ __forceinline__ void apply_twiddles_seq(c32 (&v)[R], c32 w1)
{
    if constexpr (R > 1) {
        c32 w = w1;
        v[1] = cmul(v[1], w);
        static_for<2, R>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            w = cmul(w, w1);
            v[r] = cmul(v[r], w);
        });
    }
}

// schedule options
enum : int {
    OPT_NO_PREFETCH = 1,   // fetch each group when it is processed (fewer live registers)
    OPT_SEQ_TWIDDLE = 2,   // sequential twiddle powers
    OPT_PAIRED_IO = 4,     // first/last pass: a thread owns two adjacent butterflies (16-byte I/O)
    OPT_NT = 8,            // non-temporal hint on the streaming HBM loads and stores
    OPT_EARLY_FETCH = 16,  // prefetch each pass-0 row of the next group as soon as its DFT is done
};

template <int OPT, int R>
__device__ __forceinline__ void twiddle(c32 (&v)[R], c32 w1)
{
    // The base root is loop-invariant across blocks; without this empty asm the
    // compiler hoists all R-1 powers out of the block loop and keeps them live
    // (spilling).  It emits no instruction.
    asm volatile("" : "+v"(w1.x), "+v"(w1.y));
    if constexpr (OPT & OPT_SEQ_TWIDDLE) apply_twiddles_seq<R>(v, w1);
    else apply_twiddles<R>(v, w1);
}

// Butterflies of pass p handled by one thread.  Plain: j = tid + i TB.  With
// OPT_PAIRED_IO the first and last passes give each thread two adjacent
// butterflies, j = 2 (tid + (i/2) TB) + (i%2), so their HBM accesses pair up
// into 16-byte loads and stores.
template <class PL, int TB, int OPT>
struct Map {
    static constexpr bool paired(int p) { return (OPT & OPT_PAIRED_IO) && (p == 0 || p == PL::count - 1); }
    static constexpr int nb(int p) { return PL::total() / PL::get(p); }
    static constexpr int it(int p)
    {
        return paired(p) ? 2 * ((nb(p) + 2 * TB - 1) / (2 * TB)) : (nb(p) + TB - 1) / TB;
    }
    static constexpr bool full(int p) { return paired(p) ? (it(p) * TB == nb(p)) : (it(p) * TB == nb(p)); }
    template <int P>
    __device__ static __forceinline__ int j(int tid, int i)
    {
        if constexpr (paired(P)) return 2 * (tid + (i >> 1) * TB) + (i & 1);
        else return tid + i * TB;
    }
};

// register slots of the base twiddles held by one thread: pass p >= 1 owns
// Map::it(p) consecutive slots
template <class PL, int TB, int OPT = 0>
struct TwSlots {
    static constexpr int it(int p) { return Map<PL, TB, OPT>::it(p); }
    static constexpr int off(int p)
    {
        int o = 0;
        for (int q = 1; q < p; ++q) o += it(q);
        return o;
    }
    static constexpr int total() { return PL::count > 1 ? off(PL::count) : 1; }
};

// ------------------------------------------------------------------ buffer I/O
// HBM traffic goes through raw buffer instructions on a resource that covers
// exactly the valid blocks of the current group: the per-radix offsets become
// scalar offsets (one address VGPR per thread), and accesses past the valid
// range read 0 / are dropped by the hardware range check.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <int AUX = 0>
__device__ __forceinline__ c32 ld_c(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX));
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
struct c32x2 {
    c32 a, b;
};

template <int AUX = 0>
__device__ __forceinline__ c32x2 ld_c2(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(c32x2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
}

template <int AUX = 0>
__device__ __forceinline__ float ld_f(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int AUX = 0>
__device__ __forceinline__ void st_c(c32 v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, AUX);
}

// 16-byte store.  A buffer store of more than 8 bytes needs a wait state before
// its data VGPRs are rewritten; the ISA exempts stores whose offset sits in an
// SGPR, and the compiler relies on that exemption, but on gfx950 such stores
// lost data under load when the next VALU instructions rewrote their source
// registers.  The whole offset therefore goes into the VGPR operand (opaque to
// the optimiser, so it cannot be split back into an SGPR) with a zero SGPR
// offset, and the compiler's hazard check inserts the wait state.
template <int AUX = 0>
__device__ __forceinline__ void st_c2(c32 a, c32 b, rsrc_t r, uint32_t voff, uint32_t soff)
{
    uint32_t vo = voff + soff;
    asm volatile("" : "+v"(vo));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, c32x2{a, b}), r, vo, 0, AUX);
}

struct f32x2 {
    float a, b;
};

__device__ __forceinline__ f32x2 ld_f2(rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <int AUX = 0>
__device__ __forceinline__ void st_f(float v, rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, voff, soff, AUX);
}

// ------------------------------------------------------------------ element ops
// filter factor: Lambda_n, or 1/(N Lambda_n) (v_rcp, 1 ulp; Inf for a zero tap)
__device__ __forceinline__ float filter_factor(float t, int div, float Nf)
{
    const float r = __builtin_amdgcn_rcpf(Nf * t);
    return div ? r : t;
}

// filter factors of a register array of taps, in place: the division (inverse
// side) is a wave-uniform branch on `div`, so the multiplying directions skip
// the reciprocal and the zero-tap test altogether.  `row(i)` says whether row i
// holds loaded taps (rows past the butterfly count are never loaded).
template <int A, int B, class Row>
__device__ __forceinline__ void tap_factors(float (&t)[A][B], int div, float Nf, bool &zero_tap, Row row)
{
    if (div) {
#pragma unroll
        for (int i = 0; i < A; ++i) {
            const bool ok = row(i);
#pragma unroll
            for (int r = 0; r < B; ++r) {
                zero_tap |= ok && (t[i][r] == 0.0f);
                t[i][r] = __builtin_amdgcn_rcpf(Nf * t[i][r]);
            }
        }
    }
}

// ------------------------------------------------------------------ LDS passes
// passes P <= p < END (default: all but the last) in place in LDS
template <class PL, int TB, int P, int OPT = 0, int END = PL::count - 1>
__device__ __forceinline__ void lds_passes(c32 *L, int tid, const c32 *w1s)
{
    if constexpr (P < END) {
        constexpr int N = PL::total();
        constexpr int R = PL::get(P);
        constexpr int NS = PL::ns(P);
        constexpr int NB = N / R;
        constexpr int IT = (NB + TB - 1) / TB;
        constexpr int SLOT = P == 0 ? 0 : TwSlots<PL, TB, OPT>::off(P);
        c32 v[IT][R];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = tid + i * TB;
            if (IT * TB == NB || j < NB) {
                static_for<0, R>([&](auto rI) {
                    constexpr int r = decltype(rI)::value;
                    v[i][r] = L[j + r * NB];
                });
                if constexpr (NS > 1) twiddle<OPT, R>(v[i], w1s[SLOT + i]);
                dft<R>(v[i]);
            }
        }
        lds_barrier();
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int j = tid + i * TB;
            if (IT * TB == NB || j < NB) {
                const int jm = j % NS;
                const int base = (j / NS) * NS * R + jm;
                static_for<0, R>([&](auto rI) {
                    constexpr int r = decltype(rI)::value;
                    L[base + r * NS] = v[i][r];
                });
            }
        }
        lds_barrier();
        lds_passes<PL, TB, P + 1, OPT, END>(L, tid, w1s);
    }
}

// SIDE: where the filter applies (and the exponent sign); TGR: with the tap gradient
template <class PL, int TB, int BPW, int SIDE, bool TGR, int OPT>
__global__ void __launch_bounds__(TB *BPW) fused_kernel(FusedArgs a)
{
    constexpr int TG = !TGR ? 0 : (SIDE == SIDE_OUT ? 1 : 2);
    constexpr int TG_OUT_ = 1, TG_IN_ = 2;
    constexpr int N = PL::total();
    constexpr int NP = PL::count;
    constexpr int R0 = PL::get(0);
    constexpr int NB0 = N / R0;
    using MP = Map<PL, TB, OPT>;
    constexpr int IT0 = MP::it(0);
    constexpr int RL = PL::get(NP - 1);
    constexpr int NSL = PL::ns(NP - 1);
    constexpr int NBL = N / RL;
    constexpr int ITL = MP::it(NP - 1);
    constexpr bool FULL0 = IT0 * TB == NB0;
    constexpr bool FULLL = ITL * TB == NBL;
    constexpr bool PAIR0 = MP::paired(0) && NP > 1;
    constexpr bool PAIRL = MP::paired(NP - 1) && NP > 1;
    constexpr int NACC = TG == TG_OUT_ ? ITL * RL : (TG == TG_IN_ ? IT0 * R0 : 1);
    constexpr bool CONJ = SIDE == SIDE_OUT;
    constexpr uint32_t CB = 8;      // bytes per complex
    constexpr uint32_t FB = 4;      // bytes per tap
    constexpr int NTA = (OPT & OPT_NT) ? 2 : 0;   // cache policy of the streaming accesses
    static_assert(!(OPT & OPT_PAIRED_IO) || NP > 1, "paired I/O needs at least two passes");
    static_assert(!PAIR0 || NB0 % 2 == 0, "paired I/O needs an even butterfly count");
    static_assert(!PAIRL || NBL % 2 == 0, "paired I/O needs an even butterfly count");

    __shared__ c32 lds[NP > 1 ? BPW * N : 1];
    poison_lds(lds, NP > 1 ? BPW * N : 1);
    const int bi = threadIdx.x / TB;
    const int tid = threadIdx.x - bi * TB;
    c32 *L = lds + (NP > 1 ? bi * N : 0);
    const float Nf = float(N);
    const bool shared_taps = (a.tap_stride == 0);
    const int64_t ngroups = (a.nblocks + BPW - 1) / BPW;
    // element offset of this thread's block inside its group
    const uint32_t boff = uint32_t(bi) * N;

    bool zero_tap = false;
    float acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0f;

    // base twiddles of every pass >= 1, held for the whole kernel
    c32 w1s[TwSlots<PL, TB, OPT>::total()];
    if constexpr (NP > 1) {
        static_for<1, NP>([&](auto pI) {
            constexpr int P = decltype(pI)::value;
            constexpr int NB = N / PL::get(P);
            constexpr int IT = TwSlots<PL, TB, OPT>::it(P);
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const int j = MP::template j<P>(tid, i);
                w1s[TwSlots<PL, TB, OPT>::off(P) + i] =
                    (j < NB) ? a.tw[PL::tw_off(P) + j % PL::ns(P)] : c32{1.f, 0.f};
            }
        });
    }

    // resources over the valid blocks of group g
    auto group_blocks = [&](int64_t g) -> uint32_t {
        const int64_t left = a.nblocks - g * BPW;
        return uint32_t(left < BPW ? left : BPW);
    };
    auto rs_cplx = [&](const c32 *base, int64_t g) {
        return make_rsrc(base + g * BPW * N, group_blocks(g) * N * CB);
    };
    auto rs_taps = [&](int64_t g) {
        return shared_taps ? make_rsrc(a.taps, N * FB)
                           : make_rsrc(a.taps + g * BPW * N, group_blocks(g) * N * FB);
    };

    // pass-0 operands of the group being processed: raw input and input-side taps
    c32 x0[IT0][R0];
    float t0[SIDE == SIDE_IN ? IT0 : 1][SIDE == SIDE_IN ? R0 : 1];
    // row i of group g (with paired I/O: rows i and i + 1, i even)
    auto fetch_row = [&](int64_t g, int i) {
        const rsrc_t ri = rs_cplx(a.in, g);
        const rsrc_t rt = rs_taps(g);
        const uint32_t tb = shared_taps ? 0u : boff;
        const int j = MP::template j<0>(tid, i);
        if (FULL0 || j < NB0) {
            static_for<0, R0>([&](auto rI) {
                constexpr int r = decltype(rI)::value;
                if constexpr (PAIR0) {
                    const c32x2 p = ld_c2<NTA>(ri, (boff + j) * CB, r * NB0 * CB);
                    x0[i][r] = p.a;
                    x0[i + 1][r] = p.b;
                    if constexpr (SIDE == SIDE_IN) {
                        const f32x2 t = ld_f2(rt, (tb + j) * FB, r * NB0 * FB);
                        t0[i][r] = t.a;
                        t0[i + 1][r] = t.b;
                    }
                } else {
                    x0[i][r] = ld_c<NTA>(ri, (boff + j) * CB, r * NB0 * CB);
                    if constexpr (SIDE == SIDE_IN) t0[i][r] = ld_f(rt, (tb + j) * FB, r * NB0 * FB);
                }
            });
        }
    };
    auto fetch = [&](int64_t g) {
#pragma unroll
        for (int i = 0; i < IT0; i += PAIR0 ? 2 : 1) fetch_row(g, i);
    };

    constexpr bool PREFETCH = !(OPT & OPT_NO_PREFETCH);
    // early: row i of the next group is requested right after row i's pass-0 DFT (its registers
    // are free from then on), so the CU has loads in flight during the rest of pass 0
    constexpr bool EARLY = PREFETCH && (OPT & OPT_EARLY_FETCH) && NP > 1;
    int64_t g = blockIdx.x;
    if (PREFETCH && g < ngroups) fetch(g);
    for (; g < ngroups; g += gridDim.x) {
        if (!PREFETCH) fetch(g);
        const rsrc_t ro = rs_cplx(a.out, g);
        const rsrc_t rt = rs_taps(g);
        const uint32_t tb = shared_taps ? 0u : boff;
        // this thread's block slot holds a block of the batch (the last group may be partial;
        // the taps of empty slots read as 0 and must not count as zero taps)
        const bool bvalid = uint32_t(bi) < group_blocks(g);
        rsrc_t rx = ro, rg = ro;
        if constexpr (TG != 0) {
            rx = rs_cplx(a.aux, g);
            rg = shared_taps ? ro : make_rsrc(a.tapbar + g * BPW * N, group_blocks(g) * N * FB);
        }

        if constexpr (NP == 1) {
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (FULL0 || j < NB0) {
                    c32 v[R0];
                    static_for<0, R0>([&](auto rI) {
                        constexpr int r = decltype(rI)::value;
                        if constexpr (TG == TG_IN_) {
                            const c32 s = ld_c(rx, (boff + j) * CB, r * NB0 * CB);
                            const float tg = -(x0[i][r].x * s.x + x0[i][r].y * s.y) / t0[i][r];
                            if (shared_taps) acc[i * R0 + r] += tg;
                            else st_f(tg, rg, (boff + j) * FB, r * NB0 * FB);
                        }
                        if constexpr (SIDE == SIDE_IN) {
                            zero_tap |= bvalid && (t0[i][r] == 0.0f);
                            v[r] = scale(x0[i][r], filter_factor(t0[i][r], a.div, Nf));
                        } else {
                            v[r] = conj(x0[i][r]);
                        }
                    });
                    dft<R0>(v);
                    static_for<0, R0>([&](auto rI) {
                        constexpr int r = decltype(rI)::value;
                        c32 w = CONJ ? conj(v[r]) : v[r];
                        if constexpr (TG == TG_OUT_) {
                            const c32 s = ld_c(rx, (boff + j) * CB, r * NB0 * CB);
                            const float tg = s.x * w.x + s.y * w.y;
                            if (shared_taps) acc[i * R0 + r] += tg;
                            else st_f(tg, rg, (boff + j) * FB, r * NB0 * FB);
                        }
                        if constexpr (SIDE == SIDE_OUT) {
                            const float t = ld_f(rt, (tb + j) * FB, r * NB0 * FB);
                            zero_tap |= bvalid && (t == 0.0f);
                            w = scale(w, filter_factor(t, a.div, Nf));
                        }
                        st_c(w, ro, (boff + j) * CB, r * NB0 * CB);
                    });
                }
            }
            if (PREFETCH && g + gridDim.x < ngroups) fetch(g + gridDim.x);
        } else {
            // ---- pass 0 on the fetched operands: filter, length-R0 DFT (no twiddle, Ns = 1)
            if constexpr (SIDE == SIDE_IN && TG != TG_IN_)
                tap_factors(t0, a.div, Nf, zero_tap,
                            [&](int i) { return bvalid && (FULL0 || MP::template j<0>(tid, i) < NB0); });
            c32 v0[IT0][R0];
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = MP::template j<0>(tid, i);
                if (FULL0 || j < NB0) {
                    static_for<0, R0>([&](auto rI) {
                        constexpr int r = decltype(rI)::value;
                        if constexpr (TG == TG_IN_) {
                            const c32 s = ld_c(rx, (boff + j) * CB, r * NB0 * CB);
                            const float tg = -(x0[i][r].x * s.x + x0[i][r].y * s.y) / t0[i][r];
                            if (shared_taps) acc[i * R0 + r] += tg;
                            else st_f(tg, rg, (boff + j) * FB, r * NB0 * FB);
                            zero_tap |= bvalid && (t0[i][r] == 0.0f);
                            v0[i][r] = scale(x0[i][r], filter_factor(t0[i][r], a.div, Nf));
                        } else if constexpr (SIDE == SIDE_IN) {
                            v0[i][r] = scale(x0[i][r], t0[i][r]);
                        } else {
                            v0[i][r] = conj(x0[i][r]);
                        }
                    });
                    dft<R0>(v0[i]);
                }
                if constexpr (EARLY) {
                    if (g + gridDim.x < ngroups && (!PAIR0 || (i & 1))) fetch_row(g + gridDim.x, PAIR0 ? i - 1 : i);
                }
            }
            lds_barrier();   // the previous group's last pass has finished reading LDS
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = MP::template j<0>(tid, i);
                if (FULL0 || j < NB0) {
                    static_for<0, R0>([&](auto rI) {
                        constexpr int r = decltype(rI)::value;
                        L[j * R0 + r] = v0[i][r];
                    });
                }
            }
            // ---- start reading the next group while this one runs in LDS, and the
            //      operands the last pass needs (output-side taps, S for the tap term)
            if (PREFETCH && !EARLY && g + gridDim.x < ngroups) fetch(g + gridDim.x);
            float tl[SIDE == SIDE_OUT ? ITL : 1][SIDE == SIDE_OUT ? RL : 1];
            c32 sl[TG == TG_OUT_ ? ITL : 1][TG == TG_OUT_ ? RL : 1];
#pragma unroll
            for (int i = 0; i < ITL; ++i) {
                const int j = MP::template j<NP - 1>(tid, i);
                if (FULLL || j < NBL) {
                    static_for<0, RL>([&](auto rI) {
                        constexpr int r = decltype(rI)::value;
                        if constexpr (SIDE == SIDE_OUT) tl[i][r] = ld_f(rt, (tb + j) * FB, r * NSL * FB);
                        if constexpr (TG == TG_OUT_) sl[i][r] = ld_c(rx, (boff + j) * CB, r * NSL * CB);
                    });
                }
            }
            lds_barrier();

            // ---- middle passes in LDS
            lds_passes<PL, TB, 1, OPT>(L, tid, w1s);

            // ---- last pass: LDS -> registers -> twiddle -> DFT_RL -> HBM
            if constexpr (SIDE == SIDE_OUT)
                tap_factors(tl, a.div, Nf, zero_tap,
                            [&](int i) { return bvalid && (FULLL || MP::template j<NP - 1>(tid, i) < NBL); });
            constexpr int SLOTL = TwSlots<PL, TB, OPT>::off(NP - 1);
            constexpr int STEP = PAIRL ? 2 : 1;
#pragma unroll
            for (int i = 0; i < ITL; i += STEP) {
                const int j = MP::template j<NP - 1>(tid, i);
                if (FULLL || j < NBL) {
                    c32 v[STEP][RL];
#pragma unroll
                    for (int h = 0; h < STEP; ++h) {
                        static_for<0, RL>([&](auto rI) {
                            constexpr int r = decltype(rI)::value;
                            v[h][r] = L[j + h + r * NBL];
                        });
                        twiddle<OPT, RL>(v[h], w1s[SLOTL + i + h]);
                        dft<RL>(v[h]);
                    }
                    static_for<0, RL>([&](auto rI) {
                        constexpr int r = decltype(rI)::value;
                        c32 w[STEP];
#pragma unroll
                        for (int h = 0; h < STEP; ++h) {
                            w[h] = CONJ ? conj(v[h][r]) : v[h][r];
                            if constexpr (TG == TG_OUT_) {
                                const float tg = sl[i + h][r].x * w[h].x + sl[i + h][r].y * w[h].y;
                                if (shared_taps) acc[(i + h) * RL + r] += tg;
                                else st_f(tg, rg, (boff + j + h) * FB, r * NSL * FB);
                            }
                            if constexpr (SIDE == SIDE_OUT) w[h] = scale(w[h], tl[i + h][r]);
                        }
                        if constexpr (PAIRL) st_c2<NTA>(w[0], w[1], ro, (boff + j) * CB, r * NSL * CB);
                        else st_c<NTA>(w[0], ro, (boff + j) * CB, r * NSL * CB);
                    });
                }
            }
        }
    }

    if (zero_tap && a.div && a.status) *a.status = 1;

    // ---- shared taps: one partial row of the tap gradient per (workgroup, block slot)
    if constexpr (TG != 0) {
        if (shared_taps) {
            float *row = a.tapbar + (int64_t(blockIdx.x) * BPW + bi) * N;
            if constexpr (TG == TG_IN_ || NP == 1) {
#pragma unroll
                for (int i = 0; i < IT0; ++i) {
                    const int j = MP::template j<0>(tid, i);
                    if (FULL0 || j < NB0) {
#pragma unroll
                        for (int r = 0; r < R0; ++r) row[j + r * NB0] = acc[i * R0 + r];
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < ITL; ++i) {
                    const int j = MP::template j<NP - 1>(tid, i);
                    if (FULLL || j < NBL) {
#pragma unroll
                        for (int r = 0; r < RL; ++r) row[j + r * NSL] = acc[i * RL + r];
                    }
                }
            }
        }
    }
}


// ------------------------------------------------------------------ registry entry
typedef hipError_t (*fused_launch_fn)(const FusedArgs &, unsigned grid, hipStream_t);

struct FusedEntry {
    int K, M, TB, BPW, npass, opt;
    int radix[8];
    int tw_entries;
    int lds_bytes;
    fused_launch_fn launch[2][2];     // [side][with tap gradient]
    const void *kernel[2][2];         // for occupancy queries
};

template <class PL, int TB, int BPW, int SIDE, bool TGR, int OPT>
hipError_t fused_launch(const FusedArgs &a, unsigned grid, hipStream_t s)
{
    hipLaunchKernelGGL((fused_kernel<PL, TB, BPW, SIDE, TGR, OPT>), dim3(grid), dim3(TB * BPW), 0, s, a);
    return hipGetLastError();
}

template <class PL, int TB, int BPW, int OPT = 0>
FusedEntry make_entry(int K, int M)
{
    static_assert(PL::total() <= 16384, "block too large");
    static_assert(PL::count <= 8, "too many passes");
    FusedEntry e{};
    e.K = K;
    e.M = M;
    e.TB = TB;
    e.BPW = BPW;
    e.npass = PL::count;
    for (int i = 0; i < PL::count && i < 8; ++i) e.radix[i] = PL::get(i);
    e.tw_entries = PL::tw_total();
    e.lds_bytes = PL::count > 1 ? BPW * PL::total() * (int)sizeof(c32) : 0;
    e.opt = OPT;
    e.launch[0][0] = &fused_launch<PL, TB, BPW, SIDE_IN, false, OPT>;
    e.launch[0][1] = &fused_launch<PL, TB, BPW, SIDE_IN, true, OPT>;
    e.launch[1][0] = &fused_launch<PL, TB, BPW, SIDE_OUT, false, OPT>;
    e.launch[1][1] = &fused_launch<PL, TB, BPW, SIDE_OUT, true, OPT>;
    e.kernel[0][0] = reinterpret_cast<const void *>(&fused_kernel<PL, TB, BPW, SIDE_IN, false, OPT>);
    e.kernel[0][1] = reinterpret_cast<const void *>(&fused_kernel<PL, TB, BPW, SIDE_IN, true, OPT>);
    e.kernel[1][0] = reinterpret_cast<const void *>(&fused_kernel<PL, TB, BPW, SIDE_OUT, false, OPT>);
    e.kernel[1][1] = reinterpret_cast<const void *>(&fused_kernel<PL, TB, BPW, SIDE_OUT, true, OPT>);
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
