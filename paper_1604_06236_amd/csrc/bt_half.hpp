// Block transform for K = 1024 with half-block LDS exchanges: the per-block body of the ragged
// kernel's largest class, (K, M) = (1024, 15).
//
// The operator and the pass structure are those of the uniform fused kernel with the radix plan
// [M, 32, 32]: pass 0 is the fold of eq. (7) (length-M DFT over n = p + K r, with the filter
// applied on load), passes 1 and 2 form the length-1024 IDFT with its coset twiddles, and pass 2
// writes y in natural order.  The uniform kernel keeps the whole block (8 M KB) in LDS between
// passes, so for M = 15 one block occupies a CU.  Here each exchange between two passes goes
// through a buffer of N/2 points in two rounds: a 512-thread workgroup needs 4 M KB of LDS and at
// most 128 VGPRs per thread, so two workgroups share a CU.
//
// Element e of an exchange is written by one butterfly of the pass before and read by one
// butterfly of the pass after.  Each round moves the elements of one parity class; the classes
// are chosen so that every thread writes half of its outputs and reads half of its inputs in each
// round (then no thread holds more than one butterfly's worth of values):
//   * into pass 1 (B1 = 32 M butterflies j, inputs e = j + B1 r'): round r' mod 2, slot
//     j + B1 (r' / 2).  Pass-0 butterfly p writes e = M p + r (r < M), all in round (p / 32) mod 2;
//     thread t owns p = 64 (t / 32) + t mod 32 (round 0) and p + 32 (round 1), both of which land
//     in slots M t + r.
//   * into pass 2 (e = 32 M a + M b + c with a = e / (32 M), b = (e mod 32 M) / M, c = e mod M):
//     round (a + b) mod 2, slot 16 M a + M (b / 2) + c.  Pass-1 butterfly j = M a1 + c1 writes its
//     output r at a = a1, b = r, c = c1; pass-2 butterfly j reads its input r' at a = r', b = a1,
//     c = c1.  Both pick their half by the parity of a1, which varies from lane to lane.
// Pass-1 and pass-2 butterfly j belong to thread j (32 M <= 512 threads); threads past 32 M only
// take part in pass 0.  Since each round into pass 2 delivers the inputs of one parity, pass 2's
// 32-point DFT runs as 2 x 16: each round's 16 inputs get their twiddles and a 16-point DFT as
// soon as they arrive, and the two halves are combined with one radix-2 step (the half holding
// the even inputs is selected per lane by the same bit masks).
#pragma once

#include "bt_fused.hpp"

namespace bt {

// b where the mask is set, else a, bit by bit.  The mask is opaque to the optimiser: a select
// between two elements of one register array would otherwise become a load from a computed
// address, which keeps the whole array in scratch memory.
__device__ __forceinline__ c32 blend(c32 a, c32 b, uint32_t m)
{
    const uint32_t ax = __builtin_bit_cast(uint32_t, a.x), ay = __builtin_bit_cast(uint32_t, a.y);
    const uint32_t bx = __builtin_bit_cast(uint32_t, b.x), by = __builtin_bit_cast(uint32_t, b.y);
    return c32{__builtin_bit_cast(float, (ax & ~m) | (bx & m)), __builtin_bit_cast(float, (ay & ~m) | (by & m))};
}

// Materialises the values of v at this point: the scheduler may not sink the arithmetic that
// produces them past the next barrier, where it would overlap the following exchange round and
// raise register pressure past the 128-VGPR budget.  Emits no instruction.
template <int R>
__device__ __forceinline__ void pin(c32 (&v)[R])
{
#pragma unroll
    for (int r = 0; r < R; ++r) asm volatile("" : "+v"(v[r].x), "+v"(v[r].y));
}

// LDS element as two floats (a whole-struct copy moves it as one 64-bit integer, and the float
// accesses of the transform then keep the destination array out of registers)
__device__ __forceinline__ c32 lds_get(const c32 *p) { return c32{p->x, p->y}; }

// Per-thread constants of the half-exchange body (thread t of the 512 that own one block).
// Threads past 32 M compute passes 1 and 2 on the last butterfly's operands (no branch around
// the passes, whose arrays would then stay live across the block loop) but write neither LDS
// nor HBM.
template <int M>
struct HalfThread {
    static constexpr int B1 = 32 * M;   // butterflies of passes 1 and 2
    uint32_t pa, pb;                     // pass-0 butterflies (written in rounds 0 and 1)
    int t, j;                            // thread, pass-1/2 butterfly
    bool has1;
    uint32_t odd_mask;                   // all ones where j / M is odd
    int wbase, rbase;                    // exchange into pass 2: write slot + M s, read slot + 16 M r'
    c32 w1, w2;                          // base roots of passes 1 and 2
    // w1 = exp(+2 pi i (j mod M) / (32 M)), w2 = exp(+2 pi i j / (1024 M)), read from a table
    // at the given entries (the tables of the radix plans [M, 32, 32] and [M, 8, 8, 16] both
    // hold them)
    __device__ void init(int t_, const c32 *tw1, int w1_stride, const c32 *tw2)
    {
        t = t_;
        pa = 64 * (t >> 5) + (t & 31);
        pb = pa + 32;
        has1 = t < B1;
        j = has1 ? t : B1 - 1;
        const int a1 = j / M, c1 = j - (j / M) * M;
        odd_mask = (a1 & 1) ? ~0u : 0u;
        asm volatile("" : "+v"(odd_mask));
        wbase = 16 * M * a1 + c1;
        rbase = M * (a1 >> 1) + c1;
        w1 = tw1[w1_stride * (j % M)];
        w2 = tw2[j];
    }
};

// One block: pass 0 (filter on the input side, length-M DFT), the exchange into pass 1, pass 1
// (twiddle, length-32 DFT), the exchange into pass 2 with the two 16-point halves of pass 2,
// their radix-2 combination and the natural-order store.  L
// holds N/2 points; every thread of the 512 calls it (it contains workgroup barriers).
// `valid` is false for an empty block slot (its resources have range 0: loads read 0, stores
// are dropped), whose zero taps do not count.  TAP_NT: streaming cache policy for the taps (per
// block taps; shared ones stay cached).  TGR (output side only): also store the per-block tap
// gradient Re(conj(S) y~) of the unfiltered output y~ into rg, with S read from rx.
template <int M, int SIDE, bool TAP_NT, bool TGR = false>
__device__ __forceinline__ void half_block(const HalfThread<M> &h, c32 *L, rsrc_t ri, rsrc_t ro, rsrc_t rt,
                                           rsrc_t rx, rsrc_t rg, int div, bool valid, bool &zero_tap)
{
    constexpr int K = 1024;
    constexpr int N = K * M;
    constexpr int B1 = HalfThread<M>::B1;
    constexpr uint32_t CB = 8, FB = 4;
    constexpr int NTA = 2;              // non-temporal policy of the streamed data
    constexpr int NTT = TAP_NT ? 2 : 0;
    constexpr bool CONJ = SIDE == SIDE_OUT;
    static_assert(B1 <= 512, "one pass-1 butterfly per thread");
    static_assert(!TGR || SIDE == SIDE_OUT, "tap gradient on the output side only");
    const float Nf = float(N);
    const int t = h.t, j = h.j;

    // ---- pass 0: filter (input side), length-M DFT over r for p = pa and p = pb
    c32 u[2][M];
    float tin[SIDE == SIDE_IN ? 2 : 1][SIDE == SIDE_IN ? M : 1];
    static_for<0, M>([&](auto rI) {
        constexpr int r = decltype(rI)::value;
        u[0][r] = ld_c<NTA>(ri, h.pa * CB, r * K * CB);
        u[1][r] = ld_c<NTA>(ri, h.pb * CB, r * K * CB);
        if constexpr (SIDE == SIDE_IN) {
            tin[0][r] = ld_f<NTT>(rt, h.pa * FB, r * K * FB);
            tin[1][r] = ld_f<NTT>(rt, h.pb * FB, r * K * FB);
        }
    });
    if constexpr (SIDE == SIDE_IN) tap_factors(tin, div, Nf, zero_tap, [&](int) { return valid; });
    static_for<0, 2>([&](auto hI) {
        constexpr int q = decltype(hI)::value;
        static_for<0, M>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            if constexpr (SIDE == SIDE_IN) u[q][r] = scale(u[q][r], tin[q][r]);
            else u[q][r] = conj(u[q][r]);
        });
        dft<M>(u[q]);
        pin(u[q]);
    });

    // ---- exchange into pass 1: round g carries the inputs r' = 2 s + g
    c32 v[32];
    static_for<0, 2>([&](auto gI) {
        constexpr int g = decltype(gI)::value;
        lds_barrier();   // the previous round's (or block's) reads are done
        static_for<0, M>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            L[M * t + r] = u[g][r];
        });
        lds_barrier();
        static_for<0, 16>([&](auto sI) {
            constexpr int s = decltype(sI)::value;
            v[2 * s + g] = lds_get(&L[j + B1 * s]);
        });
    });

    // ---- pass 1; its outputs in the order the exchange sends them
    twiddle<0, 32>(v, h.w1);
    dft<32>(v);
    c32 x0[16], x1[16];
    static_for<0, 16>([&](auto sI) {
        constexpr int s = decltype(sI)::value;
        x0[s] = blend(v[2 * s], v[2 * s + 1], h.odd_mask);
        x1[s] = blend(v[2 * s + 1], v[2 * s], h.odd_mask);
    });

    // ---- exchange into pass 2: round g carries the outputs r with (r + a1) mod 2 = g and
    //      the inputs r' with (r' + a1) mod 2 = g.  Pass 2's 32-point DFT is split as 2 x 16
    //      over the input parity: each round's 16 inputs (one parity class) get their twiddles
    //      w2^{r'} = w2^q (w2^2)^s and a 16-point DFT as soon as they arrive.
    c32 w2 = h.w2;
    asm volatile("" : "+v"(w2.x), "+v"(w2.y));
    const c32 w2sq = cmul(w2, w2);
    c32 z0[16], z1[16];
    static_for<0, 2>([&](auto gI) {
        constexpr int g = decltype(gI)::value;
        lds_barrier();
        if (h.has1) {
            static_for<0, 16>([&](auto sI) {
                constexpr int s = decltype(sI)::value;
                if constexpr (g == 0) L[h.wbase + M * s] = x0[s];
                else L[h.wbase + M * s] = x1[s];
            });
        }
        lds_barrier();
        const int q = g ^ (h.odd_mask & 1);           // parity of this round's r'
        c32(&zg)[16] = g == 0 ? z0 : z1;
        static_for<0, 16>([&](auto sI) {
            constexpr int s = decltype(sI)::value;
            zg[s] = lds_get(&L[h.rbase + 16 * M * (2 * s + q)]);
        });
        // base w2^q: lanes with q = 1 are those with odd a1 in round 0, even a1 in round 1
        c32 tw = blend(c32{1.f, 0.f}, w2, g == 0 ? h.odd_mask : ~h.odd_mask);
        zg[0] = cmul(zg[0], tw);
        static_for<1, 16>([&](auto sI) {
            constexpr int s = decltype(sI)::value;
            tw = cmul(tw, w2sq);
            zg[s] = cmul(zg[s], tw);
        });
        dft<16>(zg);
        pin(zg);
    });

    // ---- pass 2 (rest): combine the two halves, output side, natural-order store of y[t + B1 r]
    // even inputs: z0 on lanes with even a1, z1 on the others
    c32 z[32];
    static_for<0, 16>([&](auto kI) {
        constexpr int k = decltype(kI)::value;
        const c32 e = blend(z0[k], z1[k], h.odd_mask);
        const c32 o = rot<k, 32>(blend(z1[k], z0[k], h.odd_mask));
        z[k] = e + o;
        z[k + 16] = e - o;
    });
    if constexpr (SIDE == SIDE_OUT) {
        // the taps (and S) in groups of G outputs, each group's loads issued after the previous
        // group's stores (all 32 at once would hold 32 (96) more registers next to z)
        constexpr int G = TGR ? 4 : 8;
        static_for<0, 32 / G>([&](auto gI) {
            constexpr int g = decltype(gI)::value;
            float tg[1][G];
            c32 sv[TGR ? G : 1];
            static_for<0, G>([&](auto rI) {
                constexpr int r = G * g + decltype(rI)::value;
                tg[0][r - G * g] = ld_f<NTT>(rt, uint32_t(j) * FB, r * B1 * FB);
                if constexpr (TGR) sv[r - G * g] = ld_c<NTA>(rx, uint32_t(j) * CB, r * B1 * CB);
            });
            tap_factors(tg, div, Nf, zero_tap, [&](int) { return valid && h.has1; });
            if (h.has1) {
                static_for<0, G>([&](auto rI) {
                    constexpr int r = G * g + decltype(rI)::value;
                    const c32 w = conj(z[r]);
                    if constexpr (TGR) {
                        const c32 s_ = sv[r - G * g];
                        st_f<NTA>(s_.x * w.x + s_.y * w.y, rg, uint32_t(t) * FB, r * B1 * FB);
                    }
                    st_c<NTA>(scale(w, tg[0][r - G * g]), ro, uint32_t(t) * CB, r * B1 * CB);
                });
            }
            asm volatile("" ::: "memory");
        });
    } else {
        if (h.has1) {
            static_for<0, 32>([&](auto rI) {
                constexpr int r = decltype(rI)::value;
                st_c<NTA>(z[r], ro, uint32_t(t) * CB, r * B1 * CB);
            });
        }
    }
}

} // namespace bt
