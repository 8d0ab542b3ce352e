// Ragged batches: blocks of different (K, M) in one launch.
//
// Every block is an independent instance of the transform of eq. (6) on its
// own grid (its own N = K M, filter and offset).  The plan groups blocks of
// one (K, M) class into tiles (as many blocks as fill a workgroup), cuts them
// into work items of a few same-class tiles and sorts the items by cost
// (N log2 N per block, largest first).  One launch runs one workgroup per
// item: the hardware dispatcher hands the items out in cost order as
// workgroups retire, so there is no queue in memory and the launch replays
// from a HIP graph as it is.  Each item runs its class's compiled tile body
// (radix plan, threads per block, blocks per tile) with the same pass
// machinery as the uniform kernel; within an item the next tile's inputs are
// fetched while the current tile runs its LDS passes.  Workgroups have 512
// threads, at most 128 VGPRs and at most 74 KB of LDS, so two of any class
// share a CU; the (1024, 15) class, whose whole block would take 123 KB, runs
// the half-block exchange body of bt_half.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"
#include "bt_fused.hpp"
#include "bt_half.hpp"

namespace bt {

#ifndef BT_RAGGED_RT
#define BT_RAGGED_RT 512
#endif
#ifndef BT_RAGGED_MIN_WAVES
#define BT_RAGGED_MIN_WAVES 4
#endif
constexpr int RT = BT_RAGGED_RT;  // threads per workgroup (one tile)

struct RaggedItem {
    int cls;              // class index
    int first;            // first entry in the block order
    int count;            // blocks in this chunk (tiles of BPW blocks of the class)
    int pf;               // bit d: prefetch the next tile in body d (0 input side: forward;
                          // 1 output side: inverse, adjoint; 2 adjoint with tap gradient)
};

struct RaggedArgs {
    const c32 *in;
    c32 *out;
    const float *taps;
    const c32 *aux;
    float *tapbar;
    int *status;
    const int64_t *x_off;     // per block, in the plan's order (sorted by class and cost)
    const int64_t *tap_off;
    const RaggedItem *items;
    const c32 *tw;            // concatenated base-root tables of the classes
    const int *tw_off;        // per class
    int div;
    int lds_elems;            // complex elements of the dynamic LDS (poisoned in test builds)
};

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// Chunk body of one class: `it.count` blocks (plan entries it.first ...) processed as
// tiles of up to BPW blocks, TB threads per block (TB >= 64, so a wave never
// straddles two blocks and block bases are wave-uniform).  With PF the next
// tile's inputs are fetched while the current one runs its LDS passes.
template <class PL, int TB, int BPW, int SIDE, bool TGR, bool PF>
__device__ __forceinline__ void ragged_chunk(const RaggedArgs &a, const RaggedItem &it, c32 *lds)
{
    static_assert(TB * BPW == RT, "tile must fill the workgroup");
    static_assert(TB >= 64, "a wave must stay inside one block");
    constexpr int N = PL::total();
    constexpr int NP = PL::count;
    constexpr int R0 = PL::get(0);
    constexpr int NB0 = N / R0;
    constexpr int IT0 = (NB0 + TB - 1) / TB;
    constexpr int RL = PL::get(NP - 1);
    constexpr int NSL = PL::ns(NP - 1);
    constexpr int NBL = N / RL;
    constexpr int ITL = (NBL + TB - 1) / TB;
    constexpr bool FULL0 = IT0 * TB == NB0;
    constexpr bool FULLL = ITL * TB == NBL;
    constexpr uint32_t CB = 8, FB = 4;
    constexpr bool CONJ = SIDE == SIDE_OUT;
    constexpr int OPT = OPT_SEQ_TWIDDLE;
    constexpr int NT = 2;      // non-temporal policy for the streamed operands
    const float Nf = float(N);

    // the thread index goes through an opaque move so that the per-class
    // values derived from it are computed here, not hoisted out of the queue
    // loop where every class's copies would stay live at once
    int tx = threadIdx.x;
    asm volatile("" : "+v"(tx));
    const int bi = tx / TB;
    const int tid = tx - bi * TB;
    c32 *L = lds + bi * N;
    const int ntiles = (it.count + BPW - 1) / BPW;
    bool zero_tap = false;

    c32 w1s[TwSlots<PL, TB, OPT>::total()];
    if constexpr (NP > 1) {
        const c32 *tw = a.tw + a.tw_off[it.cls];
        static_for<1, NP>([&](auto pI) {
            constexpr int P = decltype(pI)::value;
            constexpr int NB = N / PL::get(P);
            constexpr int IT = TwSlots<PL, TB, OPT>::it(P);
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                const int j = tid + i * TB;
                w1s[TwSlots<PL, TB, OPT>::off(P) + i] = (j < NB) ? tw[PL::tw_off(P) + j % PL::ns(P)] : c32{1.f, 0.f};
            }
        });
    }

    // wave-uniform resources of this thread's block in tile t (empty for idle slots)
    struct Res {
        rsrc_t in, out, taps, aux, tg;
        bool valid;
    };
    auto res = [&](int t) {
        Res r;
        // the slot is wave-uniform (a wave never straddles two blocks); taking it through
        // readfirstlane makes the validity and the resource range scalar too, so the buffer
        // instructions get their descriptors from SGPRs as they are (a per-lane range would
        // wrap every buffer access in a loop over the distinct descriptors of the wave)
        const int slot = __builtin_amdgcn_readfirstlane(t * BPW + bi);
        r.valid = slot < it.count;
        const int e = r.valid ? it.first + slot : 0;
        // the offsets are wave-uniform; the compiler may still load them into VGPRs (a vector
        // load it cannot prove unclobbered), so they are made scalar explicitly
        const int64_t xo = uniform64(a.x_off[e]);
        const int64_t to = uniform64(a.tap_off[e]);
        const uint32_t nb = r.valid ? N : 0;
        r.in = make_rsrc(a.in + xo, nb * CB);
        r.out = make_rsrc(a.out + xo, nb * CB);
        r.taps = make_rsrc(a.taps + to, nb * FB);
        r.aux = r.out;
        r.tg = r.out;
        if constexpr (TGR) {
            r.aux = make_rsrc(a.aux + xo, nb * CB);
            r.tg = make_rsrc(a.tapbar + xo, nb * FB);
        }
        return r;
    };

    c32 x0[IT0][R0];
    float t0[SIDE == SIDE_IN ? IT0 : 1][SIDE == SIDE_IN ? R0 : 1];
    auto fetch = [&](const Res &r) {
#pragma unroll
        for (int i = 0; i < IT0; ++i) {
            const int j = tid + i * TB;
            if (FULL0 || j < NB0) {
                static_for<0, R0>([&](auto rI) {
                    constexpr int q = decltype(rI)::value;
                    x0[i][q] = ld_c<NT>(r.in, j * CB, q * NB0 * CB);
                    if constexpr (SIDE == SIDE_IN) t0[i][q] = ld_f<NT>(r.taps, j * FB, q * NB0 * FB);
                });
            }
        }
    };

    Res cur = res(0);
    if (PF) fetch(cur);
    for (int t = 0; t < ntiles; ++t) {
        if (!PF) fetch(cur);
        // ---- pass 0: filter, DFT_R0
        if constexpr (SIDE == SIDE_IN && NP > 1)
            tap_factors(t0, a.div, Nf, zero_tap,
                        [&](int i) { return cur.valid && (FULL0 || tid + i * TB < NB0); });
        c32 v0[IT0][R0];
#pragma unroll
        for (int i = 0; i < IT0; ++i) {
            const int j = tid + i * TB;
            if (FULL0 || j < NB0) {
                static_for<0, R0>([&](auto rI) {
                    constexpr int q = decltype(rI)::value;
                    if constexpr (SIDE == SIDE_IN && NP > 1) {
                        v0[i][q] = scale(x0[i][q], t0[i][q]);
                    } else if constexpr (SIDE == SIDE_IN) {
                        zero_tap |= cur.valid && (t0[i][q] == 0.0f);
                        v0[i][q] = scale(x0[i][q], filter_factor(t0[i][q], a.div, Nf));
                    } else {
                        v0[i][q] = conj(x0[i][q]);
                    }
                });
                dft<R0>(v0[i]);
            }
        }
        const Res next = res(t + 1 < ntiles ? t + 1 : t);
        if constexpr (NP == 1) {
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (FULL0 || j < NB0) {
                    static_for<0, R0>([&](auto rI) {
                        constexpr int q = decltype(rI)::value;
                        c32 w = CONJ ? conj(v0[i][q]) : v0[i][q];
                        if constexpr (TGR) {
                            const c32 sv = ld_c<NT>(cur.aux, j * CB, q * NB0 * CB);
                            st_f<NT>(sv.x * w.x + sv.y * w.y, cur.tg, j * FB, q * NB0 * FB);
                        }
                        if constexpr (SIDE == SIDE_OUT) {
                            const float tv = ld_f<NT>(cur.taps, j * FB, q * NB0 * FB);
                            zero_tap |= cur.valid && (tv == 0.0f);
                            w = scale(w, filter_factor(tv, a.div, Nf));
                        }
                        st_c<NT>(w, cur.out, j * CB, q * NB0 * CB);
                    });
                }
            }
            if (PF && t + 1 < ntiles) fetch(next);
        } else {
            lds_barrier();   // the previous tile's last pass has finished reading LDS
#pragma unroll
            for (int i = 0; i < IT0; ++i) {
                const int j = tid + i * TB;
                if (FULL0 || j < NB0) {
                    static_for<0, R0>([&](auto rI) {
                        constexpr int q = decltype(rI)::value;
                        L[j * R0 + q] = v0[i][q];
                    });
                }
            }
            if (PF && t + 1 < ntiles) fetch(next);
            // operands of the last pass, fetched while the LDS passes run; where the
            // output side's operands of the whole last pass would hold more than 16 values
            // per thread across the passes (LATE), each iteration of the last pass fetches
            // its own taps before its LDS reads instead, and with the tap gradient fetches
            // its taps and S after its DFT, four outputs at a time
            constexpr bool LATE = SIDE == SIDE_OUT && ITL * RL > 16;
            constexpr bool TL = SIDE == SIDE_OUT && !LATE;
            float tl[TL ? ITL : 1][TL ? RL : 1];
            c32 sl[TGR && !LATE ? ITL : 1][TGR && !LATE ? RL : 1];
            if constexpr (!LATE) {
#pragma unroll
                for (int i = 0; i < ITL; ++i) {
                    const int j = tid + i * TB;
                    if (FULLL || j < NBL) {
                        static_for<0, RL>([&](auto rI) {
                            constexpr int q = decltype(rI)::value;
                            if constexpr (TL) tl[i][q] = ld_f<NT>(cur.taps, j * FB, q * NSL * FB);
                            if constexpr (TGR) sl[i][q] = ld_c<NT>(cur.aux, j * CB, q * NSL * CB);
                        });
                    }
                }
            }
            lds_barrier();
            lds_passes<PL, TB, 1, OPT>(L, tid, w1s);
            if constexpr (TL)
                tap_factors(tl, a.div, Nf, zero_tap,
                            [&](int i) { return cur.valid && (FULLL || tid + i * TB < NBL); });
            constexpr int SLOTL = TwSlots<PL, TB, OPT>::off(NP - 1);
#pragma unroll
            for (int i = 0; i < ITL; ++i) {
                const int j = tid + i * TB;
                if (FULLL || j < NBL) {
                    float ti[1][LATE && !TGR ? RL : 1];
                    if constexpr (LATE && !TGR) {
                        static_for<0, RL>([&](auto rI) {
                            constexpr int q = decltype(rI)::value;
                            ti[0][q] = ld_f<NT>(cur.taps, j * FB, q * NSL * FB);
                        });
                    }
                    c32 v[RL];
                    static_for<0, RL>([&](auto rI) {
                        constexpr int q = decltype(rI)::value;
                        v[q] = L[j + q * NBL];
                    });
                    twiddle<OPT, RL>(v, w1s[SLOTL + i]);
                    dft<RL>(v);
                    if constexpr (LATE && TGR) {
                        // the taps and S in groups of 4 outputs after the DFT, each group's loads
                        // issued after the previous group's stores
                        static_for<0, RL / 4>([&](auto gI) {
                            constexpr int g = decltype(gI)::value;
                            float tg[1][4];
                            c32 sg[4];
                            static_for<0, 4>([&](auto rI) {
                                constexpr int q = 4 * g + decltype(rI)::value;
                                sg[q - 4 * g] = ld_c<NT>(cur.aux, j * CB, q * NSL * CB);
                                tg[0][q - 4 * g] = ld_f<NT>(cur.taps, j * FB, q * NSL * FB);
                            });
                            tap_factors(tg, a.div, Nf, zero_tap, [&](int) { return cur.valid; });
                            static_for<0, 4>([&](auto rI) {
                                constexpr int q = 4 * g + decltype(rI)::value;
                                const c32 w = conj(v[q]);
                                st_f<NT>(sg[q - 4 * g].x * w.x + sg[q - 4 * g].y * w.y, cur.tg, j * FB, q * NSL * FB);
                                st_c<NT>(scale(w, tg[0][q - 4 * g]), cur.out, j * CB, q * NSL * CB);
                            });
                            asm volatile("" ::: "memory");
                        });
                    } else {
                        if constexpr (LATE) tap_factors(ti, a.div, Nf, zero_tap, [&](int) { return cur.valid; });
                        static_for<0, RL>([&](auto rI) {
                            constexpr int q = decltype(rI)::value;
                            c32 w = CONJ ? conj(v[q]) : v[q];
                            if constexpr (LATE) {
                                w = scale(w, ti[0][q]);
                            } else {
                                if constexpr (TGR) st_f<NT>(sl[i][q].x * w.x + sl[i][q].y * w.y, cur.tg, j * FB, q * NSL * FB);
                                if constexpr (SIDE == SIDE_OUT) w = scale(w, tl[i][q]);
                            }
                            st_c<NT>(w, cur.out, j * CB, q * NSL * CB);
                        });
                    }
                }
            }
        }
        cur = next;
    }
    if (zero_tap && a.div && a.status) *a.status = 1;
}

// The (1024, 15) class: one block per 512-thread workgroup with the half-block LDS exchange
// body (61 KB of LDS instead of 123 KB, so that two workgroups of any class share a CU).  The
// class's radix plan stays [15, 8, 8, 16] for the plan's tables: its pass-2 and pass-3 base roots
// include the roots of the [15, 32, 32] passes.
template <int M, int SIDE, bool TGR>
__device__ __forceinline__ void ragged_half(const RaggedArgs &a, const RaggedItem &it, c32 *lds)
{
    static_assert(RT == 512, "one 512-thread block per workgroup");
    constexpr int N = 1024 * M;
    constexpr uint32_t CB = 8, FB = 4;
    int tx = threadIdx.x;
    asm volatile("" : "+v"(tx));
    const c32 *tw = a.tw + a.tw_off[it.cls];
    HalfThread<M> h;
    // [M, 8, 8, 16]: pass 2 holds exp(2 pi i k / (64 M)) at tw[M + k], pass 3 exp(2 pi i k / N)
    // at tw[9 M + k]
    h.init(tx, tw + M, 2, tw + 9 * M);
    bool zero_tap = false;
    for (int q = 0; q < it.count; ++q) {
        const int e = it.first + q;
        const int64_t xo = uniform64(a.x_off[e]), to = uniform64(a.tap_off[e]);
        const rsrc_t ri = make_rsrc(a.in + xo, N * CB), ro = make_rsrc(a.out + xo, N * CB);
        const rsrc_t rt = make_rsrc(a.taps + to, N * FB);
        if constexpr (TGR)
            half_block<M, SIDE, true, true>(h, lds, ri, ro, rt, make_rsrc(a.aux + xo, N * CB),
                                            make_rsrc(a.tapbar + xo, N * FB), a.div, true, zero_tap);
        else
            half_block<M, SIDE, true>(h, lds, ri, ro, rt, ro, ro, a.div, true, zero_tap);
    }
    if (zero_tap && a.div && a.status) *a.status = 1;
}

// ------------------------------------------------------------------ class table
// radix plans of the length-K part inside the ragged kernel: radices of at
// most 16 keep the shared register allocation (the maximum over classes) low
template <int K> struct RKPlan { using type = typename KPlan<K>::type; };
template <> struct RKPlan<512> { using type = Radices<8, 8, 8>; };
template <> struct RKPlan<1024> { using type = Radices<8, 8, 16>; };

// Per-class fitting inside the 128-VGPR budget of 512-thread workgroups at two
// per CU.  CEIL rounds the threads per block up to the next power of two above
// the widest pass (fewer elements per thread); the PF_* flags say whether the
// forward / tap-gradient adjoint / plain adjoint prefetch the next tile (a
// second copy of the pass-0 operands in registers).  The specialisations keep
// CEIL where it was measured to help and drop the prefetch from the bodies
// that would otherwise spill (per-class VGPR and spill counts of the compiler,
// one class compiled at a time); (1024, 9) goes without it in every direction.
template <int K, int M> struct RTune {
    static constexpr bool CEIL = false;
    static constexpr bool PF_FWD = true, PF_TG = true, PF_ADJ = true;
};
#define BT_RTUNE(K_, M_, CEIL_, FWD_, TG_, ADJ_)                         \
    template <> struct RTune<K_, M_> {                                    \
        static constexpr bool CEIL = CEIL_;                               \
        static constexpr bool PF_FWD = FWD_, PF_TG = TG_, PF_ADJ = ADJ_;  \
    };
BT_RTUNE(64, 9, true, true, true, true)
BT_RTUNE(64, 15, false, true, false, true)
BT_RTUNE(128, 15, false, true, false, true)
BT_RTUNE(256, 15, false, true, false, true)
BT_RTUNE(512, 9, true, true, false, true)
BT_RTUNE(512, 15, true, true, false, true)
BT_RTUNE(1024, 5, false, true, false, true)
BT_RTUNE(1024, 7, false, true, false, true)
BT_RTUNE(1024, 9, false, false, false, false)
#undef BT_RTUNE

template <int K, int M>
struct RClass {
    using PL = typename PrependM<M, typename RKPlan<K>::type>::type;
    using Tune = RTune<K, M>;
    static constexpr int TB0 = Tune::CEIL ? 2 * pow2_floor(PL::max_nb() - 1) : pow2_floor(PL::max_nb());
    static constexpr int TB = TB0 < 64 ? 64 : (TB0 > RT ? RT : TB0);
    static constexpr int BPW = RT / TB;
    // default prefetch bits (bit d for body d): the bodies that are also
    // compiled with the prefetch (where it fits the register budget); plans take these unless
    // an autotuned choice turns the prefetch off
    static constexpr int pf_default()
    {
        return (Tune::PF_FWD ? 1 : 0) | (Tune::PF_ADJ ? 2 : 0) | (Tune::PF_TG ? 4 : 0);
    }
    // (1024, 15) runs the half-block exchange body
    static constexpr bool HALF = K == 1024 && M == 15;
    static constexpr int lds() { return HALF ? PL::total() / 2 * 8 : (PL::count > 1 ? BPW * PL::total() * 8 : 0); }
};

#ifndef BT_RAGGED_CLASSES
#define BT_RAGGED_CLASSES(X)                                                                          \
    X(64, 3) X(64, 5) X(64, 7) X(64, 9) X(64, 15) X(128, 3) X(128, 5) X(128, 7) X(128, 9) X(128, 15) \
    X(256, 3) X(256, 5) X(256, 7) X(256, 9) X(256, 15) X(512, 3) X(512, 5) X(512, 7) X(512, 9)      \
    X(512, 15) X(1024, 3) X(1024, 5) X(1024, 7) X(1024, 9) X(1024, 15)
#endif

// position of (K, M) in the class list (the plan's class index)
#define BT_CLASS_KM(K_, M_) K_ * 64 + M_,
constexpr int kClassKM[] = {BT_RAGGED_CLASSES(BT_CLASS_KM)};
#undef BT_CLASS_KM
constexpr int class_index(int K, int M)
{
    for (int i = 0; i < int(sizeof(kClassKM) / sizeof(kClassKM[0])); ++i)
        if (kClassKM[i] == K * 64 + M) return i;
    return -1;
}

struct ClassInfo {
    int K, M, N, TB, BPW, lds, npass, pf, half;   // pf: default prefetch bits; half: half-block body
    int radix[8];
};

static const ClassInfo *class_table(int *count)
{
    static std::vector<ClassInfo> t = [] {
        std::vector<ClassInfo> v;
#define BT_CLASS_INFO(K_, M_)                                                               \
    {                                                                                       \
        using C = RClass<K_, M_>;                                                           \
        ClassInfo c{K_, M_, K_ * M_, C::TB, C::BPW, C::lds(), C::PL::count,                 \
                    C::HALF ? 0 : C::pf_default(), C::HALF ? 1 : 0, {}};                    \
        for (int i = 0; i < C::PL::count; ++i) c.radix[i] = C::PL::get(i);                  \
        v.push_back(c);                                                                     \
    }
        BT_RAGGED_CLASSES(BT_CLASS_INFO)
#undef BT_CLASS_INFO
        return v;
    }();
    *count = (int)t.size();
    return t.data();
}

// one workgroup per work item
template <int SIDE, bool TGR>
__global__ void __launch_bounds__(RT, BT_RAGGED_MIN_WAVES) ragged_kernel(RaggedArgs a)
{
    // 16-byte alignment lets the compiler pair each thread's LDS accesses into 64-bit
    // two-address instructions (with the 4-byte alignment of the element type it issues one
    // two-dword instruction per complex value: twice the LDS instructions)
    extern __shared__ __attribute__((aligned(16))) c32 lds_dyn[];
    poison_lds(lds_dyn, a.lds_elems);
    const RaggedItem it = a.items[blockIdx.x];
    constexpr int DIR = SIDE == SIDE_IN ? 0 : (TGR ? 2 : 1);   // body index of the prefetch bits
    // one switch (a scalar compare tree) rather than a chain of tests whose merges the
    // compiler carries as predicate masks through every class
    switch (it.cls) {
#define BT_CLASS_CASE(K_, M_)                                                                      \
    case class_index(K_, M_): {                                                                    \
        using C = RClass<K_, M_>;                                                                  \
        if constexpr (C::HALF) {                                                                   \
            static_assert(std::is_same<typename C::PL, Radices<M_, 8, 8, 16>>::value, "root table"); \
            ragged_half<M_, SIDE, TGR>(a, it, lds_dyn);                                            \
        } else if constexpr ((C::pf_default() >> DIR) & 1) {                                      \
            if ((it.pf >> DIR) & 1)                                                                \
                ragged_chunk<typename C::PL, C::TB, C::BPW, SIDE, TGR, true>(a, it, lds_dyn);      \
            else                                                                                   \
                ragged_chunk<typename C::PL, C::TB, C::BPW, SIDE, TGR, false>(a, it, lds_dyn);     \
        } else {                                                                                   \
            ragged_chunk<typename C::PL, C::TB, C::BPW, SIDE, TGR, false>(a, it, lds_dyn);         \
        }                                                                                          \
        break;                                                                                     \
    }
        BT_RAGGED_CLASSES(BT_CLASS_CASE)
#undef BT_CLASS_CASE
    default:
        break;
    }
}

// ------------------------------------------------------------------ plan
struct GraphKey {
    int dir;
    const void *in, *taps, *out, *aux, *tapbar, *status;
    bool operator<(const GraphKey &o) const
    {
        return std::tie(dir, in, taps, out, aux, tapbar, status) <
               std::tie(o.dir, o.in, o.taps, o.out, o.aux, o.tapbar, o.status);
    }
};

} // namespace bt

struct tf_ragged_plan_s {
    int device = 0;
    int64_t nblocks = 0;
    int nitems = 0;
    int max_lds = 0;
    int64_t *x_off = nullptr, *tap_off = nullptr;   // in plan order
    bt::RaggedItem *items = nullptr;
    bt::c32 *tw = nullptr;
    int *tw_off = nullptr;
    hipStream_t capture_stream = nullptr;
    std::map<bt::GraphKey, hipGraphExec_t> graphs;
    std::mutex mu;
};

using namespace bt;

static int fail(const char *what, hipError_t e)
{
    set_error(what, e);
    return TF_EHIP;
}

static void plan_free(tf_ragged_plan p)
{
    if (!p) return;
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
    (void)hipFree(p->x_off);
    (void)hipFree(p->tap_off);
    (void)hipFree(p->items);
    (void)hipFree(p->tw);
    (void)hipFree(p->tw_off);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

template <class T>
static int upload_vec(const std::vector<T> &h, T **d)
{
    hipError_t e = hipMalloc(reinterpret_cast<void **>(d), std::max<size_t>(h.size(), 1) * sizeof(T));
    if (e != hipSuccess) return fail("hipMalloc(ragged plan)", e);
    if (!h.empty()) {
        e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail("hipMemcpy(ragged plan)", e);
    }
    return TF_OK;
}

static const void *ragged_kernel_ptr(int side, bool tg)
{
    if (side == SIDE_IN) return reinterpret_cast<const void *>(&ragged_kernel<SIDE_IN, false>);
    return tg ? reinterpret_cast<const void *>(&ragged_kernel<SIDE_OUT, true>)
              : reinterpret_cast<const void *>(&ragged_kernel<SIDE_OUT, false>);
}

// autotuned prefetch choices per class and body (0 input side, 1 output side, 2 output side
// with tap gradient): -1 (compiled default), 0 (off) or 1 (on, where the default is on)
static std::mutex g_pf_mu;
static std::vector<std::array<int8_t, 3>> g_pf_choice;

static int class_of(int32_t K, int32_t M)
{
    int ncls = 0;
    const ClassInfo *cls = class_table(&ncls);
    for (int c = 0; c < ncls; ++c)
        if (cls[c].K == K && cls[c].M == M) return c;
    return -1;
}

// prefetch bits of class c in effect (caller holds g_pf_mu)
static int pf_bits(int c)
{
    int ncls = 0;
    const ClassInfo *cls = class_table(&ncls);
    if (cls[c].half) return 0;   // the half-block body has no prefetch variant
    int bits = cls[c].pf;
    if (g_pf_choice.size() == size_t(ncls))
        for (int d = 0; d < 3; ++d)
            if (g_pf_choice[c][d] == 0) bits &= ~(1 << d);
    return bits;
}

extern "C" int transform_ragged_prefetch_select(int32_t K, int32_t M, int32_t body, int32_t prefetch)
{
    if (body < 0 || body > 2 || prefetch < -1 || prefetch > 1) return TF_EINVAL;
    const int c = class_of(K, M);
    if (c < 0) return TF_EUNSUPPORTED;
    int ncls = 0;
    const ClassInfo *cls = class_table(&ncls);
    // a prefetching body exists only where the compiled default prefetches
    if (prefetch == 1 && !((cls[c].pf >> body) & 1)) return TF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_pf_mu);
    if (g_pf_choice.size() != size_t(ncls)) g_pf_choice.assign(size_t(ncls), {int8_t(-1), int8_t(-1), int8_t(-1)});
    g_pf_choice[c][body] = int8_t(prefetch);
    return TF_OK;
}

extern "C" int transform_ragged_prefetch_selected(int32_t K, int32_t M, int32_t body, int32_t *prefetch)
{
    if (body < 0 || body > 2 || !prefetch) return TF_EINVAL;
    const int c = class_of(K, M);
    if (c < 0) return TF_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_pf_mu);
    *prefetch = (pf_bits(c) >> body) & 1;
    return TF_OK;
}

extern "C" int transform_ragged_plan_create(const int32_t *K, const int32_t *M, const int64_t *x_off,
                                            const int64_t *tap_off, int64_t nblocks,
                                            int64_t total_points, tf_ragged_plan *plan)
{
    return transform_ragged_plan_create_ex(K, M, x_off, tap_off, nblocks, total_points, 0, plan);
}

extern "C" int transform_ragged_plan_create_ex(const int32_t *K, const int32_t *M, const int64_t *x_off,
                                               const int64_t *tap_off, int64_t nblocks,
                                               int64_t total_points, int32_t chunk_tiles,
                                               tf_ragged_plan *plan)
{
    if (chunk_tiles < 0) return TF_EINVAL;
    if (!plan) return TF_EINVAL;
    *plan = nullptr;
    if (nblocks < 0 || total_points < 0 || (nblocks > 0 && (!K || !M || !x_off || !tap_off)))
        return TF_EINVAL;
    if (nblocks > (int64_t(1) << 30)) return TF_EUNSUPPORTED;
    int ncls = 0;
    const ClassInfo *cls = class_table(&ncls);
    std::map<std::pair<int, int>, int> cls_of;
    for (int c = 0; c < ncls; ++c) cls_of[{cls[c].K, cls[c].M}] = c;

    std::vector<std::vector<int>> members(ncls);
    for (int64_t b = 0; b < nblocks; ++b) {
        if (!supported_km(K[b], M[b])) return TF_EUNSUPPORTED;
        auto f = cls_of.find({K[b], M[b]});
        if (f == cls_of.end()) return TF_EUNSUPPORTED;
        const int64_t N = int64_t(K[b]) * M[b];
        if (x_off[b] < 0 || x_off[b] + N > total_points || tap_off[b] < 0) return TF_EINVAL;
        members[f->second].push_back(int(b));
    }
    // work items of up to `chunk_tiles` tiles of same-class blocks, sorted by cost (largest
    // first); 0 picks four (each tile after the first has its inputs fetched while the
    // previous one runs).  No item carries more than a quarter of one workgroup slot's fair
    // share of the batch's points (slots: CUs x two workgroups), or the largest items, which
    // start first, would set the length of the launch; classes of large blocks get fewer
    // tiles per item (at least one).
    int max_lds = 0;
    for (int c = 0; c < ncls; ++c)
        if (!members[c].empty()) max_lds = std::max(max_lds, cls[c].lds);
    if (chunk_tiles == 0) chunk_tiles = 4;
    std::vector<int> order;
    std::vector<RaggedItem> items;
    std::vector<double> cost;
    std::vector<int> pf(ncls, 0);
    {
        std::lock_guard<std::mutex> lk(g_pf_mu);
        for (int c = 0; c < ncls; ++c) pf[c] = pf_bits(c);
    }
    int ncu = 0, cur_dev = 0;
    if (hipGetDevice(&cur_dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, cur_dev) != hipSuccess || ncu < 1)
        ncu = 256;
    double total_pts = 0;
    for (int c = 0; c < ncls; ++c) total_pts += double(members[c].size()) * cls[c].N;
    const double item_cap = total_pts / (double(ncu) * 2.0 * 4.0);
    for (int c = 0; c < ncls; ++c) {
        if (members[c].empty()) continue;
        const double tile_pts = double(cls[c].BPW) * cls[c].N;
        const int tiles = int(std::max(1.0, std::min(double(chunk_tiles), std::floor(item_cap / tile_pts))));
        const size_t per_chunk = size_t(cls[c].BPW) * tiles;
        for (size_t s = 0; s < members[c].size(); s += per_chunk) {
            RaggedItem it{};
            it.cls = c;
            it.pf = pf[c];
            it.first = int(order.size());
            it.count = int(std::min<size_t>(per_chunk, members[c].size() - s));
            for (int q = 0; q < it.count; ++q) order.push_back(members[c][s + q]);
            items.push_back(it);
            cost.push_back(double(it.count) * cls[c].N * std::log2(double(cls[c].N)));
        }
    }
    std::vector<int> perm(items.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = int(i);
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<RaggedItem> sorted;
    for (int i : perm) sorted.push_back(items[i]);

    // base-root twiddle tables of every class (same layout as the uniform kernel)
    std::vector<c32> tw;
    std::vector<int> tw_off(ncls, 0);
    for (int c = 0; c < ncls; ++c) {
        tw_off[c] = int(tw.size());
        long ns = cls[c].radix[0];
        for (int p = 1; p < cls[c].npass; ++p) {
            const long R = cls[c].radix[p];
            for (long jm = 0; jm < ns; ++jm) {
                const double ang = 2.0 * M_PI * double(jm) / double(ns * R);
                tw.push_back(c32{float(std::cos(ang)), float(std::sin(ang))});
            }
            ns *= R;
        }
    }

    tf_ragged_plan p = new tf_ragged_plan_s;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return TF_EHIP;
    }
    p->nblocks = nblocks;
    p->nitems = int(sorted.size());
    p->max_lds = max_lds;
    // offsets in plan order: a tile's block address is one load away from its entry
    std::vector<int64_t> xo(order.size()), to(order.size());
    for (size_t e = 0; e < order.size(); ++e) {
        xo[e] = x_off[order[e]];
        to[e] = tap_off[order[e]];
    }
    int rc = TF_OK;
    if (!rc) rc = upload_vec(xo, &p->x_off);
    if (!rc) rc = upload_vec(to, &p->tap_off);
    if (!rc) rc = upload_vec(sorted, &p->items);
    if (!rc) rc = upload_vec(tw, &p->tw);
    if (!rc) rc = upload_vec(tw_off, &p->tw_off);

    for (int v = 0; v < 3 && !rc; ++v) {
        const void *k = ragged_kernel_ptr(v == 0 ? SIDE_IN : SIDE_OUT, v == 2);
        if (max_lds > 64 * 1024) {
            hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
            if (e != hipSuccess) rc = fail("hipFuncSetAttribute", e);
        }
    }
    if (!rc) {
        hipError_t e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) rc = fail("hipStreamCreate", e);
    }
    if (rc) {
        plan_free(p);
        return rc;
    }
    *plan = p;
    return TF_OK;
}

extern "C" int transform_ragged_plan_destroy(tf_ragged_plan plan)
{
    plan_free(plan);
    return TF_OK;
}

static hipError_t ragged_launch(tf_ragged_plan p, int dir, const RaggedArgs &a, hipStream_t s)
{
    const int side = dir == 0 ? SIDE_IN : SIDE_OUT;
    const bool tg = a.tapbar != nullptr;
    RaggedArgs av = a;
    av.lds_elems = p->max_lds / int(sizeof(c32));
    const dim3 grid(p->nitems);
    if (side == SIDE_IN)
        hipLaunchKernelGGL((ragged_kernel<SIDE_IN, false>), grid, dim3(RT), p->max_lds, s, av);
    else if (tg)
        hipLaunchKernelGGL((ragged_kernel<SIDE_OUT, true>), grid, dim3(RT), p->max_lds, s, av);
    else
        hipLaunchKernelGGL((ragged_kernel<SIDE_OUT, false>), grid, dim3(RT), p->max_lds, s, av);
    return hipGetLastError();
}

extern "C" int transform_ragged_execute(tf_ragged_plan plan, int32_t direction, const void *in,
                                        const float *taps, void *out, const void *aux, float *taps_bar,
                                        int32_t *status_dev, int32_t use_graph, void *stream)
{
    if (!plan || direction < 0 || direction > 2) return TF_EINVAL;
    if (plan->nitems == 0) return TF_OK;
    if (!in || !out || !taps) return TF_EINVAL;
    if (in == out) return TF_EINVAL;
    if (taps_bar && (direction != 2 || !aux)) return TF_EINVAL;
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % 8 ||
        reinterpret_cast<uintptr_t>(taps) % 4)
        return TF_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != plan->device) return TF_EINVAL;
    RaggedArgs a{};
    a.in = reinterpret_cast<const c32 *>(in);
    a.out = reinterpret_cast<c32 *>(out);
    a.taps = taps;
    a.aux = reinterpret_cast<const c32 *>(aux);
    a.tapbar = taps_bar;
    a.status = status_dev;
    a.x_off = plan->x_off;
    a.tap_off = plan->tap_off;
    a.items = plan->items;
    a.tw = plan->tw;
    a.tw_off = plan->tw_off;
    a.div = direction == 1;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(plan->mu);
    if (!use_graph) {
        hipError_t e = ragged_launch(plan, direction, a, s);
        return e == hipSuccess ? TF_OK : fail("ragged launch", e);
    }
    GraphKey key{direction, in, taps, out, aux, taps_bar, status_dev};
    auto it = plan->graphs.find(key);
    if (it == plan->graphs.end()) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        hipError_t e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return fail("hipStreamBeginCapture", e);
        hipError_t le = ragged_launch(plan, direction, a, plan->capture_stream);
        e = hipStreamEndCapture(plan->capture_stream, &g);
        if (le != hipSuccess) return fail("ragged capture", le);
        if (e != hipSuccess) return fail("hipStreamEndCapture", e);
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail("hipGraphInstantiate", e);
        it = plan->graphs.emplace(key, ge).first;
    }
    hipError_t e = hipGraphLaunch(it->second, s);
    return e == hipSuccess ? TF_OK : fail("hipGraphLaunch", e);
}
