// Non-iterative type-5 and type-4 NFFT methods (Secs. "Computation of the
// type-5 NFFT" and "Computation of the type-4 NFFT", the type-5 and type-4 flow
// figures) on the GPU, batched over independent problems of P instants each.
//
// The non-uniform steps are exact type-1 / type-2 sums (eq. (32), eq. (34)),
// O(P R) per problem; the regular-grid steps are the block transforms of this
// library: eq. (28) is the decimated eq. (7) operator with the log-series taps
// of eq. (41), eq. (43) and eq. (31) are the inverse with the damping taps of
// eq. (8), eq. (37) is the forward with the same taps (M = 1).
//
// Numerics.  Instants are turned into 64-bit fixed-point fractions of a cycle,
// so every phase k t_q mod 1 is formed exactly in integer arithmetic before the
// sine/cosine of a remainder of at most 1/8 cycle.  The exact sums are complex
// matrix products on the FP64 matrix cores over tables of such exponentials
// (FP64 sine/cosine); the gridding kernels use an FP32 sine/cosine.  The constant phase
// P pi + 2 pi sum t of eq. (29) is likewise summed exactly as a fixed-point
// fraction.  Everything else is FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"
#include "bt_fused.hpp"

namespace bt {

constexpr int NU_MAXQ = 65536;    // instants / coefficients / frequencies per problem of the exact sums

// frac(t) as a fixed-point fraction of a cycle: T = frac(t) 2^64
__device__ __forceinline__ uint64_t fixed_instant(double t)
{
    double f = t - floor(t);
    if (!(f < 1.0)) f = 0.0;          // t just below an integer rounds up to 1.0; NaN -> 0
    return (uint64_t)(f * 18446744073709551616.0);
}

// top 32 bits of frac(k t) for an integer k >= 0: (k T mod 2^64) >> 32
__device__ __forceinline__ uint32_t phase32(uint32_t k, uint32_t tlo, uint32_t thi)
{
    return __umulhi(k, tlo) + k * thi;
}

// exp(+j 2 pi ph / 2^32).  The quadrant is split off exactly in integer
// arithmetic (nearest multiple of 2^30), leaving an angle theta of at most
// pi/4 in magnitude, whose sine and cosine are the Taylor polynomials of
// degree 9 and 8 (truncation below 2.5e-8, under one FP32 ulp of the result)
// in Horner form on theta^2.
__device__ __forceinline__ c32 cis_rev(uint32_t ph)
{
    const uint32_t quad = (ph + 0x20000000u) >> 30;              // nearest quarter cycle
    const int32_t rem = int32_t(ph - (quad << 30));               // |rem| <= 2^29
    const float th = float(rem) * 1.4629180792671596e-09f;        // 2 pi / 2^32
    const float t2 = th * th;
    const float sp = fmaf(fmaf(fmaf(fmaf(t2, 1.0f / 362880.0f, -1.0f / 5040.0f), t2, 1.0f / 120.0f), t2,
                               -1.0f / 6.0f), t2, 1.0f);
    const float s = th * sp;
    const float c = fmaf(fmaf(fmaf(fmaf(t2, 1.0f / 40320.0f, -1.0f / 720.0f), t2, 1.0f / 24.0f), t2, -0.5f),
                         t2, 1.0f);
    // rotate by quad quarter turns without branching: odd quarters swap the
    // parts, quarters 1 and 2 negate the real part, 2 and 3 the imaginary part
    const bool odd = quad & 1u;
    const float x = odd ? s : c, y = odd ? c : s;
    const uint32_t nx = ((quad + 1u) & 2u) << 30, ny = (quad & 2u) << 30;
    return c32{__uint_as_float(__float_as_uint(x) ^ nx), __uint_as_float(__float_as_uint(y) ^ ny)};
}

// ------------------------------------------------------------------ type-1 sums
// out[b][r] = sum_{q<Q} amp[b][q] exp(-j 2 pi r t[b][q]),  r < R  (eq. (32));
// amp == nullptr means unit amplitudes (the delta train z(t) of eq. (14)).

// exp(+j 2 pi ph / 2^64) in FP64: quadrant split off exactly in integers, the
// remainder theta (at most pi/4) through the Taylor polynomials of degree 13 (sine)
// and 14 (cosine); the first omitted terms are below 2.1e-14 and 1.1e-15
struct d2 {
    double x, y;
};

__device__ __forceinline__ d2 cis_rev64(uint64_t ph)
{
    const uint64_t quad = (ph + (uint64_t(1) << 61)) >> 62;
    const int64_t rem = int64_t(ph - (quad << 62));                    // |rem| <= 2^61
    const double th = double(rem) * 3.4061215800865545e-19;             // 2 pi / 2^64
    const double t2 = th * th;
    double sp = 1.0 / 6227020800.0;                                     // 1/13!
    sp = fma(sp, t2, -1.0 / 39916800.0);
    sp = fma(sp, t2, 1.0 / 362880.0);
    sp = fma(sp, t2, -1.0 / 5040.0);
    sp = fma(sp, t2, 1.0 / 120.0);
    sp = fma(sp, t2, -1.0 / 6.0);
    const double sn = th * fma(sp, t2, 1.0);
    double cp = -1.0 / 87178291200.0;                                   // -1/14!
    cp = fma(cp, t2, 1.0 / 479001600.0);
    cp = fma(cp, t2, -1.0 / 3628800.0);
    cp = fma(cp, t2, 1.0 / 40320.0);
    cp = fma(cp, t2, -1.0 / 720.0);
    cp = fma(cp, t2, 1.0 / 24.0);
    cp = fma(cp, t2, -0.5);
    const double cs = fma(cp, t2, 1.0);
    const bool odd = quad & 1u;
    const double x = odd ? sn : cs, y = odd ? cs : sn;
    const bool nx = (quad + 1u) & 2u, ny = quad & 2u;
    return d2{nx ? -x : x, ny ? -y : y};
}

__device__ __forceinline__ d2 cmul64(d2 a, d2 b) { return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

typedef double dd4 __attribute__((ext_vector_type(4)));

// Complex products on the FP64 matrix cores, three real products per complex one
// (Gauss): with the A tile stored as (re, im, re + im) and the B tile as
// (re, im - re, re + im),  T1 = (Ar + Ai) Br,  T2 = Ar (Bi - Br),  T3 = Ai (Br + Bi),
// re = T1 - T3,  im = T1 + T2.  v_mfma_f64_16x16x4 operand layout (lane l):
// A[l % 16][l / 16], B[l / 16][l % 16], result element j at D[4 j + l / 16][l % 16].
struct cacc {
    dd4 t1, t2, t3;
};

__device__ __forceinline__ void cmfma(cacc &d, double as, double ar, double ai, double br, double bd, double bs)
{
    d.t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(as, br, d.t1, 0, 0, 0);
    d.t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bd, d.t2, 0, 0, 0);
    d.t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bs, d.t3, 0, 0, 0);
}

constexpr int NU_QC = 16;    // contraction depth staged per step of the matrix-core sums

// Type-1 sum as a complex matrix product.  With r = r1 + 64 r2,
// A(r) = sum_q U[r1][q] V[q][r2],  U[r1][q] = a_q e^{-j 2 pi r1 t_q},
// V[q][r2] = e^{-j 2 pi 64 r2 t_q}: the O(Q R) phase evaluations of the direct sum
// become O(Q (64 + R/64)) table entries (exact 64-bit fixed-point phases, FP64
// sine/cosine) and the sum itself runs on the matrix cores.  One workgroup per
// (problem, 16 CT columns of r2) with G groups of four waves; group g takes every
// G-th chunk of 16 instants (more waves per CU when a problem has few columns), and
// the groups' partial sums are added through LDS at the end.  Wave w of a group owns
// the rows r1 in [16 w, 16 w + 16).  R is padded to a multiple of 64; the extra
// outputs are computed and dropped.  With NBUF = 2 the tables of the next chunk are
// built while the matrix cores work on the current one (one barrier per chunk).
template <int CT, int G, int NBUF>
struct Nu1Smem {
    static constexpr int NC = 16 * CT;
    struct Tab {
        double u[2][64][NU_QC + 1];     // a e^{-j 2 pi r1 t}: re, im
        double v[2][NU_QC][NC + 1];     // e^{-j 2 pi 64 r2 t}: re, im
    };
    union {
        Tab tab[G][NBUF];
        double red[G > 1 ? G - 1 : 1][4][G > 1 ? CT : 1][2][4][64];    // group sums (G > 1 only)
    };
};

template <int CT, int G, int NBUF, int MINW = 1>
__global__ void __launch_bounds__(256 * G, MINW) nudft1_mfma_kernel(const double *t, const c32 *amp, c32 *out, int Q, int R)
{
    using Sm = Nu1Smem<CT, G, NBUF>;
    using Tab = typename Sm::Tab;
    __shared__ Sm sm;
    const int64_t b = blockIdx.y;
    const int R2 = (R + 63) / 64;       // columns; outputs r >= R of the last one are not stored
    const int c0 = blockIdx.x * Sm::NC;
    const int g = threadIdx.x >> 8, tx = threadIdx.x & 255;
    const int w = tx >> 6, l = tx & 63;
    cacc acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct].t1 = acc[ct].t2 = acc[ct].t3 = dd4{0.0, 0.0, 0.0, 0.0};

    // tables of chunk `it` of this group: thread (qq, i0) fills the rows r1 = i0 + 16 i
    // and the columns j = i0 + 16 i of instant qq, each run from one exponential and
    // its step e^{-j 2 pi 16 r t}
    auto build = [&](int it, Tab &tb) {
        const int qq = tx & 15, i0 = tx >> 4;
        const int q = (it * G + g) * NU_QC + qq;
        const bool live = q < Q;
        const uint64_t T = live ? fixed_instant(t[b * Q + q]) : 0;
        const c32 a = live ? (amp ? amp[b * Q + q] : c32{1.f, 0.f}) : c32{0.f, 0.f};
        const double ax = a.x, ay = a.y;
        d2 c = cis_rev64(uint64_t(0) - uint64_t(i0) * T);                        // e^{-j 2 pi r1 t}
        c = d2{ax * c.x - ay * c.y, ax * c.y + ay * c.x};
        // the steps e^{-j 2 pi 16 t} and e^{-j 2 pi 1024 t} are shared by the four lanes of a
        // wave that hold instant qq (lanes qq, qq + 16, qq + 32, qq + 48): one exponential per
        // lane, then broadcast
        const int lane = tx & 63;
        const d2 se = cis_rev64(uint64_t(0) - uint64_t((lane >> 4) == 1 ? 1024 : 16) * T);
        const d2 st = d2{__shfl(se.x, lane & 15), __shfl(se.y, lane & 15)};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            tb.u[0][i0 + 16 * i][qq] = c.x;
            tb.u[1][i0 + 16 * i][qq] = c.y;
            if (i < 3) c = cmul64(c, st);
        }
        d2 v = cis_rev64(uint64_t(0) - uint64_t(64 * (c0 + i0)) * T);             // e^{-j 2 pi 64 r2 t}
        const d2 sv = d2{__shfl(se.x, (lane & 15) + 16), __shfl(se.y, (lane & 15) + 16)};
#pragma unroll
        for (int i = 0; i < CT; ++i) {
            const int j = i0 + 16 * i;
            const bool on = live && c0 + j < R2;
            tb.v[0][qq][j] = on ? v.x : 0.0;
            tb.v[1][qq][j] = on ? v.y : 0.0;
            if (i + 1 < CT) v = cmul64(v, sv);
        }
    };
    auto contract = [&](const Tab &tb) {
#pragma unroll
        for (int s4 = 0; s4 < NU_QC / 4; ++s4) {
            const int kq = 4 * s4 + (l >> 4), row = 16 * w + (l & 15);
            const double ar = tb.u[0][row][kq], ai = tb.u[1][row][kq];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = 16 * ct + (l & 15);
                const double br = tb.v[0][kq][col], bi = tb.v[1][kq][col];
                cmfma(acc[ct], ar + ai, ar, ai, br, bi - br, br + bi);
            }
        }
    };

    const int nit = (Q + G * NU_QC - 1) / (G * NU_QC);      // the same trip count for every group
    if constexpr (NBUF == 1) {
        for (int it = 0; it < nit; ++it) {
            build(it, sm.tab[g][0]);
            __syncthreads();
            contract(sm.tab[g][0]);
            __syncthreads();
        }
    } else {
        if (nit > 0) build(0, sm.tab[g][0]);
        __syncthreads();
        for (int it = 0; it < nit; ++it) {
            // buffer (it + 1) & 1 was last read in the previous chunk, before its barrier
            if (it + 1 < nit) build(it + 1, sm.tab[g][(it + 1) & 1]);
            contract(sm.tab[g][it & 1]);
            __syncthreads();
        }
    }
    if constexpr (G > 1) {
        // the tables are dead (last barrier above): reuse their LDS for the group sums
        if (g > 0) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sm.red[g - 1][w][ct][0][j][l] = acc[ct].t1[j] - acc[ct].t3[j];
                    sm.red[g - 1][w][ct][1][j][l] = acc[ct].t1[j] + acc[ct].t2[j];
                }
        }
        __syncthreads();
        if (g > 0) return;
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int r2 = c0 + 16 * ct + (l & 15);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            double re = acc[ct].t1[j] - acc[ct].t3[j], im = acc[ct].t1[j] + acc[ct].t2[j];
#pragma unroll
            for (int h = 0; h + 1 < G; ++h) {
                re += sm.red[h][w][ct][0][j][l];
                im += sm.red[h][w][ct][1][j][l];
            }
            const int r = 16 * w + 4 * j + (l >> 4) + 64 * r2;
            if (r < R) out[b * R + r] = c32{float(re), float(im)};
        }
    }
}

// ------------------------------------------------------------------ type-2 sums
// out[b][q] = sum_{p<P} c_p exp(+j 2 pi p t[b][q]),  q < Q  (eq. (34)).
// deriv == 0: c_p = coef[b][p].  deriv == 1: the coefficients of L'(z) from the
// P lower coefficients of the monic L (eq. (16)): c_p = (p+1) coef[b][p+1] for
// p < P-1, c_{P-1} = P (L_P = 1).

// Type-2 sum on the matrix cores.  With p = p1 + 64 p2,
// s(t_q) = sum_{p1<64} e^{j 2 pi p1 t_q} W[p1][q],  W[p1][q] = sum_{p2} C[p1][p2] V[p2][q],
// C[p1][p2] = c_{p1 + 64 p2},  V[p2][q] = e^{j 2 pi 64 p2 t_q}:  W is a complex matrix
// product over ceil(P/64) terms (16 per staged step, zero-padded), the outer sum a
// pointwise product with a 64-row reduction.  One workgroup of four waves per
// (problem, 16 CT instants); wave w owns the rows p1 in [16 w, 16 w + 16).
// Coefficients c_p as described above (deriv: those of L', eq. (16)).
template <int CT>
__global__ void __launch_bounds__(256, CT > 2 ? 2 : 4) nudft2_mfma_kernel(const double *t, const c32 *coef, c32 *out, int P, int Q,
                                                         int deriv)
{
    constexpr int NC = 16 * CT;
    constexpr int KS = 256 / NC;                // V-table rows one thread steps over
    static_assert(256 % NC == 0 && NU_QC % KS == 0, "V-table fill assumes NC | 256");
    __shared__ double cu[2][64][NU_QC + 1];     // C: re, im
    __shared__ double vb[2][NU_QC][NC + 1];     // V: re, im
    __shared__ uint64_t sT[NC];
    __shared__ double red[2][4][NC];
    const int64_t b = blockIdx.y;
    const int P2 = (P + 63) / 64;      // coefficients p >= P of the last column are zero
    const int c0 = blockIdx.x * NC;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (threadIdx.x < NC) {
        const int q = c0 + threadIdx.x;
        sT[threadIdx.x] = q < Q ? fixed_instant(t[b * Q + q]) : 0;
    }
    cacc acc[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[ct].t1 = acc[ct].t2 = acc[ct].t3 = dd4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    for (int k0 = 0; k0 < P2; k0 += NU_QC) {
        for (int e = threadIdx.x; e < 64 * NU_QC; e += 256) {
            const int kk = e / 64, p1 = e % 64;          // consecutive threads: consecutive coefficients
            const int p = p1 + 64 * (k0 + kk);
            double cr = 0.0, ci = 0.0;
            if (p < P) {
                if (!deriv) {
                    const c32 c = coef[b * P + p];
                    cr = c.x;
                    ci = c.y;
                } else if (p + 1 < P) {
                    const c32 c = coef[b * P + p + 1];
                    cr = double(p + 1) * c.x;
                    ci = double(p + 1) * c.y;
                } else {
                    cr = double(P);
                }
            }
            cu[0][p1][kk] = cr;
            cu[1][p1][kk] = ci;
        }
        {
            // e^{j 2 pi 64 p2 t} for p2 = k0 + kk: a thread owns one instant j and the rows
            // kk0, kk0 + KS, ...; one exponential for the first row, one for the step
            const int j = threadIdx.x % NC, kk0 = threadIdx.x / NC;
            const uint64_t T = sT[j];
            d2 c = cis_rev64(uint64_t(64 * (k0 + kk0)) * T);
            const d2 st = cis_rev64(uint64_t(64 * KS) * T);
#pragma unroll
            for (int i = 0; i < NU_QC / KS; ++i) {
                const int kk = kk0 + i * KS;
                const bool live = k0 + kk < P2;
                vb[0][kk][j] = live ? c.x : 0.0;
                vb[1][kk][j] = live ? c.y : 0.0;
                c = cmul64(c, st);
            }
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < NU_QC / 4; ++s4) {
            const int kq = 4 * s4 + (l >> 4), row = 16 * w + (l & 15);
            const double ar = cu[0][row][kq], ai = cu[1][row][kq];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = 16 * ct + (l & 15);
                const double br = vb[0][kq][col], bi = vb[1][kq][col];
                cmfma(acc[ct], ar + ai, ar, ai, br, bi - br, br + bi);
            }
        }
        __syncthreads();
    }
    // outer sum: e^{j 2 pi p1 t_q} W[p1][q] over the lane's four rows, then over the
    // four row groups of the wave (lanes l, l ^ 16, l ^ 32, l ^ 48) and the four waves.
    // The four lanes of a column (k4 = l / 16) share their exponentials: each evaluates
    // one of e^{j 2 pi m t}, m = 16 w, 1, 2, 4, and the others arrive by shuffle.
    const int k4 = l >> 4, c16 = l & 15;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int col = 16 * ct + c16;
        const uint64_t T = sT[col];
        double re = 0.0, im = 0.0;
        const uint64_t m = k4 == 0 ? uint64_t(16 * w) : uint64_t(1) << ((k4 + 3) & 3);
        const d2 e = cis_rev64(m * T);
        const d2 e0 = d2{__shfl(e.x, c16), __shfl(e.y, c16)};
        const d2 e1 = d2{__shfl(e.x, c16 + 16), __shfl(e.y, c16 + 16)};
        const d2 e2 = d2{__shfl(e.x, c16 + 32), __shfl(e.y, c16 + 32)};
        const d2 su = d2{__shfl(e.x, c16 + 48), __shfl(e.y, c16 + 48)};   // e^{j 2 pi 4 t}
        d2 u = (k4 & 1) ? cmul64(e0, e1) : e0;
        if (k4 & 2) u = cmul64(u, e2);                                   // e^{j 2 pi p1 t}, p1 = 16 w + 4 j + k4
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double wr = acc[ct].t1[j] - acc[ct].t3[j], wi = acc[ct].t1[j] + acc[ct].t2[j];
            re += u.x * wr - u.y * wi;
            im += u.x * wi + u.y * wr;
            if (j < 3) u = cmul64(u, su);
        }
        re += __shfl_xor(re, 16);
        im += __shfl_xor(im, 16);
        re += __shfl_xor(re, 32);
        im += __shfl_xor(im, 32);
        if (l < 16) {
            red[0][w][col] = re;
            red[1][w][col] = im;
        }
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        const int q = c0 + threadIdx.x;
        const double re = red[0][0][threadIdx.x] + red[0][1][threadIdx.x] + red[0][2][threadIdx.x] +
                          red[0][3][threadIdx.x];
        const double im = red[1][0][threadIdx.x] + red[1][1][threadIdx.x] + red[1][2][threadIdx.x] +
                          red[1][3][threadIdx.x];
        if (q < Q) out[b * Q + q] = c32{float(re), float(im)};
    }
}

// ------------------------------------------------------------------ pointwise steps
// g of eq. (41) (R taps) and the damping filter exp(-2 pi p a) of eq. (8) (P taps)
__global__ void nufft_taps_kernel(float *g, int R, float *damp, int P, double a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double two_pi = 6.283185307179586476925286766559;
    if (i < R) g[i] = (i == 0) ? 0.f : float(-exp(-two_pi * a * double(i)) / double(i));
    if (i < P) damp[i] = float(exp(-two_pi * a * double(i)));
}

// kernel samples eq. (29): Lk_q = exp(j P pi + j 2 pi sum_p t_p + v_q); one
// workgroup per problem, the constant phase summed exactly in fixed point
template <int TPB>
__global__ void __launch_bounds__(TPB) nufft_kernel_samples(const double *t, const c32 *v, c32 *Lk, int P)
{
    __shared__ uint64_t s_sum[TPB];
    const int64_t b = blockIdx.x;
    uint64_t acc = 0;
    for (int q = threadIdx.x; q < P; q += TPB) acc += fixed_instant(t[b * P + q]);
    s_sum[threadIdx.x] = acc;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
        __syncthreads();
    }
    // P pi = 2 pi (P / 2): half a cycle when P is odd
    const uint64_t c0 = s_sum[0] + ((P & 1) ? (uint64_t(1) << 63) : 0);
    const double rev0 = double(c0 >> 11) * 0x1p-53;                 // in [0, 1)
    const double inv_two_pi = 0.15915494309189533576888376337251;
    for (int q = threadIdx.x; q < P; q += TPB) {
        const c32 vq = v[b * P + q];
        double rev = rev0 + double(vq.y) * inv_two_pi;
        rev -= rint(rev);                                            // [-1/2, 1/2]
        float s, c;
        sincospif(float(2.0 * rev), &s, &c);
        const float m = expf(vq.x);
        Lk[b * P + q] = c32{m * c, m * s};
    }
}

// delta-train weights, eq. (27) / eq. (40):
//   out_q = x_q h(-P t_q + j P a) / (L'(e^{j 2 pi t_q}) e^{j 2 pi t_q}),
//   h(-P t + j P a) = 1 / (rho e^{-j 2 pi P t} - 1),  rho = e^{-2 pi P a}
__global__ void nufft_weights_kernel(const double *t, const c32 *Ld, const c32 *x, c32 *out, int P,
                                     int64_t total, float rho)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const uint64_t T = fixed_instant(t[i]);
    const uint32_t lo = uint32_t(T), hi = uint32_t(T >> 32);
    const c32 eP = cis_rev(0u - phase32(uint32_t(P), lo, hi));     // e^{-j 2 pi P t}
    const c32 e1 = cis_rev(hi);                                      // e^{+j 2 pi t}
    const c32 hd = c32{rho * eP.x - 1.f, rho * eP.y};               // 1 / h
    const c32 d = Ld[i];
    const c32 de = c32{d.x * e1.x - d.y * e1.y, d.x * e1.y + d.y * e1.x};
    const c32 den = c32{hd.x * de.x - hd.y * de.y, hd.x * de.y + hd.y * de.x};
    const float inv = 1.f / (den.x * den.x + den.y * den.y);
    const c32 xv = x[i];
    out[i] = c32{(xv.x * den.x + xv.y * den.y) * inv, (xv.y * den.x - xv.x * den.y) * inv};
}

// element-wise product, eq. (30)
__global__ void nufft_cmul_kernel(const c32 *a, const c32 *b, c32 *out, int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const c32 x = a[i], y = b[i];
    out[i] = c32{x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x};
}

// y += alpha x (residual and correction of the refinement, eq. (44)-(46))
__global__ void nufft_axpy_kernel(c32 *y, const c32 *x, float alpha, int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const c32 a = y[i], b = x[i];
    y[i] = c32{a.x + alpha * b.x, a.y + alpha * b.y};
}

// ------------------------------------------------------------------ gridding NFFTs
// Type-1 / type-2 NFFTs by gridding at oversampling 2 with the Gaussian window of
// Dutt-Rokhlin / Greengard-Lee: fine grid n = 2 (band size),
// g(x) = exp(-x^2 / (4 tau)) periodised, tau = ln(1/eps) / (2 pi^2 n^2), kept on
// the 2 GRID_HALF grid points around n t, g_hat(k) = sqrt(4 pi tau) exp(-4 pi^2 k^2 tau).
// The band 0..R-1 of eq. (32) is the centred band -R/2..R/2-1 after a modulation
// by exp(-j 2 pi (R/2) t); the FFTs are this library's transforms with the
// deconvolution 1 / g_hat folded into their taps.  eps = 1e-7 (FP32 level).
constexpr int GRID_HALF = 8;                         // ceil(sqrt(2) ln(1e7) / pi)
constexpr double GRID_LOG_INV_EPS = 16.11809565095832;   // ln(1e7)

// spread the (modulated) amplitudes of one problem onto its fine grid, then store
// the grid.  One workgroup per problem.  The accumulation is in 64-bit fixed
// point with LDS integer atomics (the float LDS atomics of this chip are several
// times slower, and integer sums are exact and order-independent): every
// product c w is a float whose scaling by 2^S is exact, with 2^S chosen from the
// largest amplitude so that Q max|a| 2^S < 2^62; each sum is rounded once, when
// it is converted back to FP32.  Real and imaginary parts take one pass each, so
// the LDS grid is n 64-bit words (dynamic LDS).
template <int TPB>
__global__ void __launch_bounds__(TPB) grid_spread_kernel(const double *t, const c32 *amp, c32 *grid, int Q, int n,
                                                          int rhalf, float kappa)
{
    extern __shared__ unsigned long long g_acc[];
    __shared__ float s_max[TPB / 64];
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    // scale: the modulation has unit magnitude, so |Re c|, |Im c| <= |a|
    float mx = 0.f;
    for (int q = threadIdx.x; q < Q; q += TPB) {
        const c32 a = amp ? amp[b * Q + q] : c32{1.f, 0.f};
        mx = fmaxf(mx, fmaxf(fabsf(a.x), fabsf(a.y)));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) s_max[wv] = mx;
    __syncthreads();
    mx = 0.f;
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) mx = fmaxf(mx, s_max[i]);
    int e_a = 0, e_q = 0;
    frexpf(mx, &e_a);                            // mx < 2^e_a
    frexpf(float(Q), &e_q);                      // Q < 2^e_q (or equal: then 2^e_q > Q)
    const int S = mx > 0.f ? 62 - e_a - e_q : 0;
    const float up = ldexpf(1.0f, S), down = ldexpf(1.0f, -S);

    float *gf = reinterpret_cast<float *>(grid + b * n);
    for (int comp = 0; comp < 2; ++comp) {
        for (int i = threadIdx.x; i < n; i += TPB) g_acc[i] = 0ull;
        __syncthreads();
        for (int q = threadIdx.x; q < Q; q += TPB) {
            const uint64_t T = fixed_instant(t[b * Q + q]);
            const c32 a = amp ? amp[b * Q + q] : c32{1.f, 0.f};
            const c32 e = cis_rev(0u - phase32(uint32_t(rhalf), uint32_t(T), uint32_t(T >> 32)));
            const float cv = comp == 0 ? a.x * e.x - a.y * e.y : a.x * e.y + a.y * e.x;
            const double x = double(T >> 11) * 0x1p-53 * double(n);        // n t in [0, n)
            const double fl = floor(x);
            const int m0 = min(int(fl), n - 1);
            const float fx = float(x - fl);
            for (int j = -GRID_HALF + 1; j <= GRID_HALF; ++j) {
                int m = m0 + j;
                m = m < 0 ? m + n : (m >= n ? m - n : m);
                const float d = fx - float(j);
                const float w = __expf(-kappa * d * d);
                const long long v = (long long)((cv * w) * up);           // exact: a power-of-two scaling
                atomicAdd(&g_acc[m], (unsigned long long)v);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += TPB) gf[2 * i + comp] = float((long long)g_acc[i]) * down;
        __syncthreads();
    }
}

// deconvolution taps over the n bins of the fine grid: for the bins of the
// centred band -band/2..band/2-1, scale / g_hat(k); zero elsewhere
__global__ void grid_taps_kernel(float *taps, int n, int band, double tau, double scale)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = i < n / 2 ? i : i - n;
    const double pi = 3.14159265358979323846;
    const bool in_band = k >= -(band / 2) && k < band - band / 2;
    taps[i] = in_band ? float(scale * exp(4.0 * pi * pi * double(k) * double(k) * tau) / sqrt(4.0 * pi * tau))
                      : 0.f;
}

// band 0..R-1 from the fine-grid spectrum: out[b][r] = spec[b][(r - R/2) mod n]
__global__ void grid_pick_kernel(const c32 *spec, c32 *out, int R, int n, int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t b = i / R;
    const int r = int(i - b * R);
    int k = r - R / 2;
    if (k < 0) k += n;
    out[i] = spec[b * n + k];
}

// coefficients 0..P-1 onto the fine-grid bins of the centred band (zeros
// elsewhere); deriv = 1 builds the coefficients of L' from L (eq. (16))
__global__ void grid_load_kernel(const c32 *coef, c32 *H, int P, int n, int deriv, int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t b = i / n;
    const int bin = int(i - b * n);
    const int k = bin < n / 2 ? bin : bin - n;
    const int p = k + P / 2;
    c32 v = c32{0.f, 0.f};
    if (p >= 0 && p < P) {
        if (!deriv) {
            v = coef[b * P + p];
        } else if (p + 1 < P) {
            const c32 l = coef[b * P + p + 1];
            v = c32{float(p + 1) * l.x, float(p + 1) * l.y};
        } else {
            v = c32{float(P), 0.f};
        }
    }
    H[i] = v;
}

// interpolation: out_q = e^{j 2 pi (P/2) t_q} (1/n) sum_j h[(m0 + j) mod n] g(t_q - (m0 + j)/n)
__global__ void grid_interp_kernel(const double *t, const c32 *h, c32 *out, int Q, int n, int phalf, float kappa,
                                   int64_t total)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t b = i / Q;
    const uint64_t T = fixed_instant(t[i]);
    const double x = double(T >> 11) * 0x1p-53 * double(n);
    const double fl = floor(x);
    const int m0 = min(int(fl), n - 1);
    const float fx = float(x - fl);
    float sx = 0.f, sy = 0.f;
    const c32 *hb = h + b * n;
    for (int j = -GRID_HALF + 1; j <= GRID_HALF; ++j) {
        int m = m0 + j;
        m = m < 0 ? m + n : (m >= n ? m - n : m);
        const float d = fx - float(j);
        const float w = __expf(-kappa * d * d);
        const c32 v = hb[m];
        sx += v.x * w;
        sy += v.y * w;
    }
    const c32 e = cis_rev(phase32(uint32_t(phalf), uint32_t(T), uint32_t(T >> 32)));
    const float inv_n = 1.f / float(n);
    out[i] = c32{(sx * e.x - sy * e.y) * inv_n, (sx * e.y + sy * e.x) * inv_n};
}

// ------------------------------------------------------------------ host side
constexpr int NU_PW_TPB = 256;

static bool nu_aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static int nu_check_launch(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(what, e);
        return TF_EHIP;
    }
    return TF_OK;
}

static int nudft1_launch(const double *t, const c32 *amp, c32 *out, int64_t nblocks, int Q, int R, hipStream_t s)
{
    // three column tiles per workgroup when the grid still fills the chip, else one
    // tile and the instants split over two or four wave groups
    const int R2 = (R + 63) / 64;
    const int64_t g3 = (R2 + 47) / 48, g1 = (R2 + 15) / 16;
    if (R2 >= 48 && g3 * nblocks >= 512) {
        hipLaunchKernelGGL((nudft1_mfma_kernel<3, 2, 1, 4>), dim3(unsigned(g3), unsigned(nblocks)), dim3(512), 0, s, t,
                           amp, out, Q, R);
    } else if (g1 * nblocks >= 1024 || Q <= 2 * NU_QC) {
        hipLaunchKernelGGL((nudft1_mfma_kernel<1, 1, 2>), dim3(unsigned(g1), unsigned(nblocks)), dim3(256), 0, s, t,
                           amp, out, Q, R);
    } else if (g1 * nblocks >= 512 || Q <= 4 * NU_QC) {
        hipLaunchKernelGGL((nudft1_mfma_kernel<1, 2, 2>), dim3(unsigned(g1), unsigned(nblocks)), dim3(512), 0, s, t,
                           amp, out, Q, R);
    } else {
        hipLaunchKernelGGL((nudft1_mfma_kernel<1, 4, 1>), dim3(unsigned(g1), unsigned(nblocks)), dim3(1024), 0, s, t,
                           amp, out, Q, R);
    }
    return nu_check_launch("nudft_type1 launch");
}

static int nudft2_launch(const double *t, const c32 *coef, c32 *out, int64_t nblocks, int P, int Q, int deriv,
                         hipStream_t s)
{
    // 64 instants per workgroup: the staged coefficients serve twice as many instants as
    // with 32, at three waves per SIMD (168 VGPRs, no spills); 2-5 % faster than 32 or 16
    hipLaunchKernelGGL((nudft2_mfma_kernel<4>), dim3(unsigned((Q + 63) / 64), unsigned(nblocks)), dim3(256), 0, s, t,
                       coef, out, P, Q, deriv);
    return nu_check_launch("nudft_type2 launch");
}

static bool nu_blocks_ok(int64_t nblocks) { return nblocks >= 1 && nblocks <= 65535; }

// fine-grid size for a band of `band` frequencies and its factorisation n = K M
// for the block transforms (K a power of two <= 1024, M <= 16)
static bool grid_shape(int band, int *n, int *K, int *M)
{
    if (band < 16 || band % 2) return false;        // the window's 16 points must fit in the period
    const int nn = 2 * band;
    int k = 1;
    while (k < 1024 && nn % (2 * k) == 0) k *= 2;
    if (nn / k > 16 || !supported_km(k, nn / k)) return false;
    *n = nn;
    *K = k;
    *M = nn / k;
    return nn <= 16384;
}

static double grid_tau(int n) { return GRID_LOG_INV_EPS / (2.0 * M_PI * M_PI * double(n) * double(n)); }
// g(d / n) = exp(-kappa d^2) for a distance of d grid cells
static float grid_kappa() { return float(M_PI * M_PI / (2.0 * GRID_LOG_INV_EPS)); }

static int grid_spread_attr()
{
    static int rc = [] {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&grid_spread_kernel<1024>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 16384 * 8);
        if (e != hipSuccess) {
            set_error("hipFuncSetAttribute(grid spread)", e);
            return int(TF_EHIP);
        }
        return int(TF_OK);
    }();
    return rc;
}

// gridding type-1: out[b][r], r < R, from Q instants; scratch: grid and spectrum
// (nblocks n complex each) and n taps
static int grid1_run(const double *t, const c32 *amp, c32 *out, int64_t nblocks, int Q, int R, c32 *grid,
                     c32 *spec, float *taps, void *stream)
{
    int n, K, M, rc;
    if (!grid_shape(R, &n, &K, &M)) return TF_EUNSUPPORTED;
    if ((rc = grid_spread_attr())) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const double tau = grid_tau(n);
    hipLaunchKernelGGL(grid_taps_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, taps, n, R, tau,
                       1.0 / double(n));
    if ((rc = nu_check_launch("grid taps launch"))) return rc;
    hipLaunchKernelGGL((grid_spread_kernel<1024>), dim3(unsigned(nblocks)), dim3(1024), size_t(n) * 8, s, t, amp,
                       grid, Q, n, R / 2, grid_kappa());
    if ((rc = nu_check_launch("grid spread launch"))) return rc;
    if ((rc = transform_adjoint(grid, taps, nullptr, spec, nullptr, nblocks, K, M, 0, TF_FP32, nullptr, 0, stream)))
        return rc;
    const int64_t total = nblocks * R;
    hipLaunchKernelGGL(grid_pick_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, spec, out, R, n,
                       total);
    return nu_check_launch("grid pick launch");
}

// gridding type-2: out[b][q], q < Q, from P coefficients (deriv: those of L')
static int grid2_run(const double *t, const c32 *coef, c32 *out, int64_t nblocks, int P, int Q, int deriv,
                     c32 *grid, c32 *spec, float *taps, void *stream)
{
    int n, K, M, rc;
    if (!grid_shape(P, &n, &K, &M)) return TF_EUNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const double tau = grid_tau(n);
    hipLaunchKernelGGL(grid_taps_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, taps, n, P, tau, 1.0);
    if ((rc = nu_check_launch("grid taps launch"))) return rc;
    const int64_t tn = nblocks * n;
    hipLaunchKernelGGL(grid_load_kernel, dim3(unsigned((tn + 255) / 256)), dim3(256), 0, s, coef, spec, P, n, deriv,
                       tn);
    if ((rc = nu_check_launch("grid load launch"))) return rc;
    if ((rc = transform_forward(spec, taps, grid, nblocks, K, M, 0, TF_FP32, nullptr, 0, stream))) return rc;
    const int64_t tq = nblocks * Q;
    hipLaunchKernelGGL(grid_interp_kernel, dim3(unsigned((tq + 255) / 256)), dim3(256), 0, s, t, grid, out, Q, n,
                       P / 2, grid_kappa(), tq);
    return nu_check_launch("grid interp launch");
}

// workspace layout, each segment 256-byte aligned
struct NuLayout {
    size_t g, damp, Z, v, Lk, Lc, Ld, t1, t2, t3, t4, gg, gs, gt, total;
};

static size_t nu_round(size_t x) { return (x + 255) & ~size_t(255); }

static NuLayout nu_layout(int64_t nblocks, int P, int eta, bool gridding = false)
{
    NuLayout l{};
    const size_t R = size_t(P) * eta, BP = size_t(nblocks) * P * sizeof(c32);
    size_t o = 0;
    l.g = o;    o += nu_round(R * sizeof(float));
    l.damp = o; o += nu_round(size_t(P) * sizeof(float));
    l.Z = o;    o += nu_round(size_t(nblocks) * R * sizeof(c32));
    l.v = o;    o += nu_round(BP);
    l.Lk = o;   o += nu_round(BP);
    l.Lc = o;   o += nu_round(BP);
    l.Ld = o;   o += nu_round(BP);
    l.t1 = o;   o += nu_round(BP);
    l.t2 = o;   o += nu_round(BP);
    l.t3 = o;   o += nu_round(BP);
    l.t4 = o;   o += nu_round(BP);
    // gridding scratch: fine grid and spectrum for the largest band (R), its taps
    const size_t nmax = gridding ? 2 * R : 0;
    l.gg = o;   o += nu_round(size_t(nblocks) * nmax * sizeof(c32));
    l.gs = o;   o += nu_round(size_t(nblocks) * nmax * sizeof(c32));
    l.gt = o;   o += nu_round(nmax * sizeof(float));
    l.total = o;
    return l;
}

static bool nu_shape_ok(int P, int eta)
{
    return P >= 16 && P <= 1024 && (P & (P - 1)) == 0 && eta >= 1 && eta <= 16;
}

struct NuBufs {
    float *g, *damp;
    c32 *Z, *v, *Lk, *Lc, *Ld, *t1, *t2, *t3, *t4;
    c32 *gg, *gs;      // gridding scratch
    float *gt;
    bool grid;         // non-uniform sums by gridding instead of exact sums
};

// the non-uniform sums of the pipeline: exact, or by gridding
static int sum1(const NuBufs &b, const double *t, const c32 *amp, c32 *out, int64_t nblocks, int Q, int R,
                void *stream)
{
    if (b.grid) return grid1_run(t, amp, out, nblocks, Q, R, b.gg, b.gs, b.gt, stream);
    return nudft1_launch(t, amp, out, nblocks, Q, R, reinterpret_cast<hipStream_t>(stream));
}

static int sum2(const NuBufs &b, const double *t, const c32 *coef, c32 *out, int64_t nblocks, int P, int Q,
                int deriv, void *stream)
{
    if (b.grid) return grid2_run(t, coef, out, nblocks, P, Q, deriv, b.gg, b.gs, b.gt, stream);
    return nudft2_launch(t, coef, out, nblocks, P, Q, deriv, reinterpret_cast<hipStream_t>(stream));
}

// the part of both methods that depends on the instants only: filters, kernel
// samples (eq. (28), eq. (29)), Lagrange coefficients (eq. (43)) and derivative
// samples (eq. (16))
static int nu_setup(const double *t, int64_t nblocks, int P, int eta, double a, const NuBufs &b, void *stream)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int R = P * eta;
    int rc;
    // filters of eq. (41) and eq. (8)
    hipLaunchKernelGGL(nufft_taps_kernel, dim3(unsigned((R + 255) / 256)), dim3(256), 0, s, b.g, R, b.damp, P, a);
    if ((rc = nu_check_launch("nufft taps launch"))) return rc;
    // eq. (28): unit delta train -> spectrum at 0..R-1 -> decimated eq. (7) with g
    if ((rc = sum1(b, t, nullptr, b.Z, nblocks, P, R, stream))) return rc;
    if ((rc = transform_decimated(b.Z, b.g, b.v, nblocks, P, eta, 0, stream))) return rc;
    // eq. (29): kernel samples on the shifted grid
    hipLaunchKernelGGL((nufft_kernel_samples<256>), dim3(unsigned(nblocks)), dim3(256), 0, s, t, b.v, b.Lk, P);
    if ((rc = nu_check_launch("nufft kernel samples launch"))) return rc;
    // eq. (43): L_p = e^{2 pi p a} DFT(Lk)_p / P for p >= 1 (the alias fix touches L_0 only,
    // which the derivative of eq. (16) never reads)
    if ((rc = transform_inverse(b.Lk, b.damp, b.Lc, nblocks, P, 1, 0, TF_FP32, nullptr, nullptr, 0, stream)))
        return rc;
    // eq. (16): L'(e^{j 2 pi t_q}) by a type-2 sum
    return sum2(b, t, b.Lc, b.Ld, nblocks, P, P, 1, stream);
}

// kind 5: x = samples s(t_q) -> y = coefficients S_p (type-5 flow)
// kind 4: x = spectral samples A(r) -> y = amplitudes a_q (type-4 flow)
static int nu_apply(int kind, const double *t, const c32 *x, c32 *y, int64_t nblocks, int P, double a,
                    const NuBufs &b, void *stream)
{
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t BP = nblocks * P;
    const unsigned pw_grid = unsigned((BP + NU_PW_TPB - 1) / NU_PW_TPB);
    const float rho = float(std::exp(-2.0 * M_PI * double(P) * a));
    int rc;
    if (kind == 5) {
        // eq. (27) weights -> type-1 sum -> eq. (37): the summation eq. (25)
        hipLaunchKernelGGL(nufft_weights_kernel, dim3(pw_grid), dim3(NU_PW_TPB), 0, s, t, b.Ld, x, b.t1, P, BP, rho);
        if ((rc = nu_check_launch("nufft weights launch"))) return rc;
        if ((rc = sum1(b, t, b.t1, b.t2, nblocks, P, P, stream))) return rc;
        if ((rc = transform_forward(b.t2, b.damp, b.t1, nblocks, P, 1, 0, TF_FP32, nullptr, 0, stream))) return rc;
        // eq. (30), then eq. (31)
        hipLaunchKernelGGL(nufft_cmul_kernel, dim3(pw_grid), dim3(NU_PW_TPB), 0, s, b.Lk, b.t1, b.t2, BP);
        if ((rc = nu_check_launch("nufft product launch"))) return rc;
        return transform_inverse(b.t2, b.damp, y, nblocks, P, 1, 0, TF_FP32, nullptr, nullptr, 0, stream);
    }
    // type 4: eq. (37) -> eq. (30) -> eq. (31) -> type-2 sum -> eq. (40)
    if ((rc = transform_forward(x, b.damp, b.t1, nblocks, P, 1, 0, TF_FP32, nullptr, 0, stream))) return rc;
    hipLaunchKernelGGL(nufft_cmul_kernel, dim3(pw_grid), dim3(NU_PW_TPB), 0, s, b.Lk, b.t1, b.t2, BP);
    if ((rc = nu_check_launch("nufft product launch"))) return rc;
    if ((rc = transform_inverse(b.t2, b.damp, b.t1, nblocks, P, 1, 0, TF_FP32, nullptr, nullptr, 0, stream)))
        return rc;
    if ((rc = sum2(b, t, b.t1, b.t2, nblocks, P, P, 0, stream))) return rc;
    hipLaunchKernelGGL(nufft_weights_kernel, dim3(pw_grid), dim3(NU_PW_TPB), 0, s, t, b.Ld, b.t2, y, P, BP, rho);
    return nu_check_launch("nufft weights launch");
}

// refine == 0: one pass of the method.  refine == 1: the refined method of
// Sec. 5 (eq. (44)-(46)): y0 = method(x); residual r = F y0 - x with F the
// forward map of the system (the type-1 sum for type 4, the type-2 evaluation
// for type 5); y = y0 - method(r).  The setup is shared by both passes.
static bool nu_grid_ok(int P, int eta)
{
    int n, K, M;
    return grid_shape(P * eta, &n, &K, &M) && grid_shape(P, &n, &K, &M);
}

// phases of a call: the setup (instants only), the application to one input, or both
enum { NU_SETUP = 1, NU_APPLY = 2 };

static int nufft_run(int kind, int flags, const double *t, const void *in, void *out, int64_t nblocks, int P,
                     int eta, double a, void *ws, size_t ws_bytes, void *stream, int phases = NU_SETUP | NU_APPLY)
{
    const bool refine = flags & NUFFT_REFINE, gridding = flags & NUFFT_GRIDDING;
    const bool apply = phases & NU_APPLY;
    if (flags & ~(NUFFT_REFINE | NUFFT_GRIDDING)) return TF_EINVAL;
    if (!nu_shape_ok(P, eta) || (gridding && !nu_grid_ok(P, eta))) return TF_EUNSUPPORTED;
    if (!(a > 0.0) || !std::isfinite(a)) return TF_EINVAL;
    if (nblocks == 0) return TF_OK;                       // an empty batch is a no-op
    if (!nu_blocks_ok(nblocks)) return TF_EINVAL;
    if (!t || !nu_aligned(t, 8)) return TF_EINVAL;
    if (apply && (!in || !out || !nu_aligned(in, 8) || !nu_aligned(out, 8))) return TF_EINVAL;
    const NuLayout l = nu_layout(nblocks, P, eta, gridding);
    if (!ws || ws_bytes < l.total || !nu_aligned(ws, 256)) return TF_EWORKSPACE;
    const size_t io_bytes = size_t(nblocks) * P * sizeof(c32);
    const uintptr_t pw = reinterpret_cast<uintptr_t>(ws), po = reinterpret_cast<uintptr_t>(out),
                    pi = reinterpret_cast<uintptr_t>(in), pt = reinterpret_cast<uintptr_t>(t);
    const size_t t_bytes = size_t(nblocks) * P * sizeof(double);
    auto ov = [](uintptr_t x, size_t xb, uintptr_t y, size_t yb) { return x < y + yb && y < x + xb; };
    if (ov(pt, t_bytes, pw, l.total)) return TF_EINVAL;
    if (apply && (ov(po, io_bytes, pw, l.total) || ov(pi, io_bytes, pw, l.total) || ov(po, io_bytes, pt, t_bytes)))
        return TF_EINVAL;
    // the refinement reads the input again after the first pass has written the output
    if (apply && refine && ov(po, io_bytes, pi, io_bytes)) return TF_EINVAL;

    char *w = static_cast<char *>(ws);
    NuBufs b;
    b.g = reinterpret_cast<float *>(w + l.g);
    b.damp = reinterpret_cast<float *>(w + l.damp);
    b.Z = reinterpret_cast<c32 *>(w + l.Z);
    b.v = reinterpret_cast<c32 *>(w + l.v);
    b.Lk = reinterpret_cast<c32 *>(w + l.Lk);
    b.Lc = reinterpret_cast<c32 *>(w + l.Lc);
    b.Ld = reinterpret_cast<c32 *>(w + l.Ld);
    b.t1 = reinterpret_cast<c32 *>(w + l.t1);
    b.t2 = reinterpret_cast<c32 *>(w + l.t2);
    b.t3 = reinterpret_cast<c32 *>(w + l.t3);
    b.t4 = reinterpret_cast<c32 *>(w + l.t4);
    b.gg = reinterpret_cast<c32 *>(w + l.gg);
    b.gs = reinterpret_cast<c32 *>(w + l.gs);
    b.gt = reinterpret_cast<float *>(w + l.gt);
    b.grid = gridding;
    const c32 *x = reinterpret_cast<const c32 *>(in);
    c32 *y = reinterpret_cast<c32 *>(out);
    int rc;
    if ((phases & NU_SETUP) && (rc = nu_setup(t, nblocks, P, eta, a, b, stream))) return rc;
    if (!apply) return TF_OK;
    if ((rc = nu_apply(kind, t, x, y, nblocks, P, a, b, stream))) return rc;
    if (!refine) return TF_OK;

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t BP = nblocks * P;
    const unsigned pw_grid = unsigned((BP + NU_PW_TPB - 1) / NU_PW_TPB);
    // residual of the first pass: F y0 - x
    if (kind == 4) rc = sum1(b, t, y, b.t3, nblocks, P, P, stream);
    else rc = sum2(b, t, y, b.t3, nblocks, P, P, 0, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(nufft_axpy_kernel, dim3(pw_grid), dim3(NU_PW_TPB), 0, s, b.t3, x, -1.f, BP);
    if ((rc = nu_check_launch("nufft residual launch"))) return rc;
    // the method on the residual, subtracted from the first pass
    if ((rc = nu_apply(kind, t, b.t3, b.t4, nblocks, P, a, b, stream))) return rc;
    hipLaunchKernelGGL(nufft_axpy_kernel, dim3(pw_grid), dim3(NU_PW_TPB), 0, s, y, b.t4, -1.f, BP);
    return nu_check_launch("nufft correction launch");
}

} // namespace bt

using namespace bt;

extern "C" size_t nufft_workspace_size(int64_t nblocks, int32_t P, int32_t eta)
{
    return nufft_workspace_size_ex(nblocks, P, eta, 0);
}

extern "C" size_t nufft_workspace_size_ex(int64_t nblocks, int32_t P, int32_t eta, int32_t flags)
{
    if (!nu_shape_ok(P, eta) || !nu_blocks_ok(nblocks)) return 0;
    if ((flags & NUFFT_GRIDDING) && !nu_grid_ok(P, eta)) return 0;
    return nu_layout(nblocks, P, eta, (flags & NUFFT_GRIDDING) != 0).total;
}

extern "C" int nufft_solve(int32_t type, int32_t flags, const double *t, const void *in, void *out, int64_t nblocks,
                           int32_t P, int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream)
{
    if (type != 4 && type != 5) return TF_EINVAL;
    return nufft_run(type, flags, t, in, out, nblocks, P, eta, a, workspace, workspace_bytes, stream);
}

extern "C" int nufft_setup(int32_t flags, const double *t, int64_t nblocks, int32_t P, int32_t eta, double a,
                           void *workspace, size_t workspace_bytes, void *stream)
{
    return nufft_run(5, flags, t, nullptr, nullptr, nblocks, P, eta, a, workspace, workspace_bytes, stream, NU_SETUP);
}

extern "C" int nufft_apply(int32_t type, int32_t flags, const double *t, const void *in, void *out, int64_t nblocks,
                           int32_t P, int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream)
{
    if (type != 4 && type != 5) return TF_EINVAL;
    return nufft_run(type, flags, t, in, out, nblocks, P, eta, a, workspace, workspace_bytes, stream, NU_APPLY);
}

extern "C" int nufft_type5(const double *t, const void *samples, void *coeffs, int64_t nblocks, int32_t P,
                           int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream)
{
    return nufft_run(5, 0, t, samples, coeffs, nblocks, P, eta, a, workspace, workspace_bytes, stream);
}

extern "C" int nufft_type4(const double *t, const void *spectrum, void *amplitudes, int64_t nblocks, int32_t P,
                           int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream)
{
    return nufft_run(4, 0, t, spectrum, amplitudes, nblocks, P, eta, a, workspace, workspace_bytes, stream);
}

extern "C" int nufft_type5_refined(const double *t, const void *samples, void *coeffs, int64_t nblocks, int32_t P,
                                   int32_t eta, double a, void *workspace, size_t workspace_bytes, void *stream)
{
    return nufft_run(5, NUFFT_REFINE, t, samples, coeffs, nblocks, P, eta, a, workspace, workspace_bytes, stream);
}

extern "C" int nufft_type4_refined(const double *t, const void *spectrum, void *amplitudes, int64_t nblocks,
                                   int32_t P, int32_t eta, double a, void *workspace, size_t workspace_bytes,
                                   void *stream)
{
    return nufft_run(4, NUFFT_REFINE, t, spectrum, amplitudes, nblocks, P, eta, a, workspace, workspace_bytes,
                     stream);
}

extern "C" size_t nfft_workspace_size(int64_t nblocks, int32_t band)
{
    int n, K, M;
    if (!nu_blocks_ok(nblocks) || !grid_shape(band, &n, &K, &M)) return 0;
    return 2 * nu_round(size_t(nblocks) * n * sizeof(c32)) + nu_round(size_t(n) * sizeof(float));
}

static int nfft_ws(int64_t nblocks, int band, void *ws, size_t ws_bytes, c32 **grid, c32 **spec, float **taps)
{
    int n, K, M;
    if (!grid_shape(band, &n, &K, &M)) return TF_EUNSUPPORTED;
    const size_t seg = nu_round(size_t(nblocks) * n * sizeof(c32));
    if (!ws || ws_bytes < nfft_workspace_size(nblocks, band) || !nu_aligned(ws, 256)) return TF_EWORKSPACE;
    char *w = static_cast<char *>(ws);
    *grid = reinterpret_cast<c32 *>(w);
    *spec = reinterpret_cast<c32 *>(w + seg);
    *taps = reinterpret_cast<float *>(w + 2 * seg);
    return TF_OK;
}

extern "C" int nfft_type1(const double *t, const void *amp, void *out, int64_t nblocks, int32_t Q, int32_t R,
                          void *workspace, size_t workspace_bytes, void *stream)
{
    if (Q < 1 || Q > 65536) return TF_EUNSUPPORTED;
    if (nblocks == 0) return TF_OK;
    if (!nu_blocks_ok(nblocks)) return TF_EUNSUPPORTED;
    if (!t || !out || !nu_aligned(t, 8) || !nu_aligned(out, 8) || (amp && !nu_aligned(amp, 8))) return TF_EINVAL;
    c32 *grid, *spec;
    float *taps;
    int rc = nfft_ws(nblocks, R, workspace, workspace_bytes, &grid, &spec, &taps);
    if (rc) return rc;
    return grid1_run(t, reinterpret_cast<const c32 *>(amp), reinterpret_cast<c32 *>(out), nblocks, Q, R, grid, spec,
                     taps, stream);
}

extern "C" int nfft_type2(const double *t, const void *coeffs, void *out, int64_t nblocks, int32_t P, int32_t Q,
                          void *workspace, size_t workspace_bytes, void *stream)
{
    if (Q < 1 || Q > 65536) return TF_EUNSUPPORTED;
    if (nblocks == 0) return TF_OK;
    if (!nu_blocks_ok(nblocks)) return TF_EUNSUPPORTED;
    if (!t || !coeffs || !out || !nu_aligned(t, 8) || !nu_aligned(coeffs, 8) || !nu_aligned(out, 8))
        return TF_EINVAL;
    c32 *grid, *spec;
    float *taps;
    int rc = nfft_ws(nblocks, P, workspace, workspace_bytes, &grid, &spec, &taps);
    if (rc) return rc;
    return grid2_run(t, reinterpret_cast<const c32 *>(coeffs), reinterpret_cast<c32 *>(out), nblocks, P, Q, 0, grid,
                     spec, taps, stream);
}

extern "C" int nudft_type1(const double *t, const void *amp, void *out, int64_t nblocks, int32_t Q, int32_t R,
                           void *stream)
{
    if (Q < 1 || Q > NU_MAXQ || R < 1 || R > NU_MAXQ) return TF_EUNSUPPORTED;
    if (nblocks == 0) return TF_OK;
    if (!nu_blocks_ok(nblocks)) return TF_EUNSUPPORTED;
    if (!t || !out || !nu_aligned(t, 8) || !nu_aligned(out, 8) || (amp && !nu_aligned(amp, 8))) return TF_EINVAL;
    return nudft1_launch(t, reinterpret_cast<const c32 *>(amp), reinterpret_cast<c32 *>(out), nblocks, Q, R,
                         reinterpret_cast<hipStream_t>(stream));
}

extern "C" int nudft_type2(const double *t, const void *coeffs, void *out, int64_t nblocks, int32_t P, int32_t Q,
                           void *stream)
{
    if (P < 1 || P > NU_MAXQ || Q < 1 || Q > NU_MAXQ) return TF_EUNSUPPORTED;
    if (nblocks == 0) return TF_OK;
    if (!nu_blocks_ok(nblocks)) return TF_EUNSUPPORTED;
    if (!t || !coeffs || !out || !nu_aligned(t, 8) || !nu_aligned(coeffs, 8) || !nu_aligned(out, 8))
        return TF_EINVAL;
    return nudft2_launch(t, reinterpret_cast<const c32 *>(coeffs), reinterpret_cast<c32 *>(out), nblocks, P, Q, 0,
                         reinterpret_cast<hipStream_t>(stream));
}
