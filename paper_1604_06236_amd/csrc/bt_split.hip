// Split-precision GEMM-DFT path: the short DFT stages of the transform run as
// matrix-core (MFMA) GEMMs on BF16 or FP16 operands with FP32 accumulation.
//
// Per block (N = K M, K = KS*KS with KS in {16, 32}), positive exponent:
//   stage A  U[m][p] = sum_{r<M} F_M[m][r] Z[r][p]       Z[r][p] = Lambda S at n = p + K r
//            (the circular fold of eq. (7), all M cosets; F_M zero-padded to 16x16)
//            U[m][p] *= e^{+j 2 pi p m / N}                 (coset twiddle)
//   stage B1 V[p1][q2] = sum_{p2} U[m][p1 + KS p2] F_KS[p2][q2]   (p = p1 + KS p2)
//            V[p1][q2] *= e^{+j 2 pi p1 q2 / K}
//   stage B2 X[q1][q2] = sum_{p1} F_KS[q1][p1] V[p1][q2]            (q = q2 + KS q1)
//   y_{M q + m} = X[q1][q2]
// which is the length-K IDFT of eq. (7) split into two KS-point DFTs.  The
// negative exponent (adjoint) conjugates inputs and outputs.
//
// Each real operand x is split into hi = round(x) and lo = round(x - hi) in the
// 16-bit format; a real product a b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi
// (three MFMAs, the lo*lo term dropped), accumulated in FP32.  FP16 operands are
// scaled by powers of two chosen from the data's magnitude so that the lo parts
// stay normal; the scales are removed exactly at the end.
//
// Layouts (gfx950, wave64): for v_mfma_f32_16x16x16 lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16]; the 16x16x32 forms take k = 8(l/16)+j.
// The k order of stage B1/B2 is permuted (slot 8g+j <-> p = 4g+j for j < 4 and
// 16+4g+j-4 otherwise) so that the D registers of B1 are the B operand of B2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/blocktransform.h"
#include "bt_api_internal.hpp"
#include "bt_dft.hpp"
#include "bt_fused.hpp"

namespace bt {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

struct PrecBF16 {
    typedef __bf16 T;
    typedef bf4 V4;
    typedef bf8 V8;
    static constexpr bool scaled = false;
    __device__ static f4 mma16(V4 a, V4 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c,
                                                         0, 0, 0);
    }
    __device__ static f4 mma32(V8 a, V8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};

struct PrecFP16 {
    typedef _Float16 T;
    typedef h4 V4;
    typedef h8 V8;
    static constexpr bool scaled = true;
    __device__ static f4 mma16(V4 a, V4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
    __device__ static f4 mma32(V8 a, V8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};

// split of a complex vector into hi/lo parts of re and im; the constant operands (the DFT
// matrices) also carry -im, so that the data operands never need a negated copy
template <class P, int W>
struct SplitC {
    typedef typename P::T T;
    typedef T V __attribute__((ext_vector_type(W)));
    V rh, rl, ih, il, nih, nil;
    __device__ void set(int j, c32 x)
    {
        const T a = T(x.x), b = T(x.y);
        rh[j] = a;
        rl[j] = T(x.x - float(a));
        ih[j] = b;
        il[j] = T(x.y - float(b));
        nih[j] = -ih[j];
        nil[j] = -il[j];
    }
};

template <class P, int W, class V>
__device__ __forceinline__ f4 mma(V a, V b, f4 c)
{
    if constexpr (W == 4) return P::mma16(a, b, c);
    else return P::mma32(a, b, c);
}

// complex tile product D += A B, A and B split; each real product with 3 MFMAs (the lo*lo term
// dropped).  NEG_A: the -Im(A) Im(B) term takes A's negated parts (A constant), else B's (B
// constant).
template <class P, int W, bool NEG_A>
__device__ __forceinline__ void cmma(const SplitC<P, W> &A, const SplitC<P, W> &B, f4 &dr, f4 &di)
{
    dr = mma<P, W>(A.rh, B.rh, dr); dr = mma<P, W>(A.rh, B.rl, dr); dr = mma<P, W>(A.rl, B.rh, dr);
    if constexpr (NEG_A) {
        dr = mma<P, W>(A.nih, B.ih, dr); dr = mma<P, W>(A.nih, B.il, dr); dr = mma<P, W>(A.nil, B.ih, dr);
    } else {
        dr = mma<P, W>(A.ih, B.nih, dr); dr = mma<P, W>(A.ih, B.nil, dr); dr = mma<P, W>(A.il, B.nih, dr);
    }
    di = mma<P, W>(A.rh, B.ih, di); di = mma<P, W>(A.rh, B.il, di); di = mma<P, W>(A.rl, B.ih, di);
    di = mma<P, W>(A.ih, B.rh, di); di = mma<P, W>(A.ih, B.rl, di); di = mma<P, W>(A.il, B.rh, di);
}

struct SplitArgs {
    const c32 *in;
    c32 *out;
    const float *taps;
    const c32 *fm;        // [16][16] e^{+j 2 pi m r / M}, zero outside m, r < M
    const c32 *fk;        // [KS][KS] e^{+j 2 pi a b / KS}
    const c32 *ta;        // [K][16]  e^{+j 2 pi p m / N}
    const c32 *tb;        // [KS][KS] e^{+j 2 pi p1 q2 / K}
    int64_t nblocks;
    int64_t tap_stride;
    int M;
};

constexpr int ST = 512;   // threads per workgroup (8 waves)

// k slot -> row index of the 32-wide chunk (see the header comment)
__device__ __forceinline__ int kperm32(int g, int j) { return j < 4 ? 4 * g + j : 16 + 4 * g + j - 4; }

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// power of two s with max * s in [2^13, 2^14); 1 for max == 0
__device__ __forceinline__ float pow2_scale(float mx)
{
    if (!(mx > 0.0f)) return 1.0f;
    int e;
    frexpf(mx, &e);                 // mx = f 2^e, f in [0.5, 1)
    return ldexpf(1.0f, 14 - e);
}

template <int KS, class P, int SIDE>
__global__ void __launch_bounds__(ST) split_kernel(SplitArgs a)
{
    constexpr int K = KS * KS;
    constexpr int NT = K / 16;                  // p tiles of stage A
    constexpr int RS = K + 1;                   // padded LDS row stride
    constexpr int KW = KS == 32 ? 8 : 4;        // k per lane in stages B1/B2
    constexpr int NKT = KS / 16;                // 16-wide tiles per KS
    __shared__ c32 U[16 * RS];
    __shared__ float red[ST / 64];

    const int M = a.M;
    const int N = K * M;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const bool conj_io = SIDE == SIDE_OUT;

    // constants: F_M in the A layout of 16x16x16, F_KS tiles in the B layout of the B stages
    SplitC<P, 4> fm;
#pragma unroll
    for (int j = 0; j < 4; ++j) fm.set(j, a.fm[c * 16 + 4 * g + j]);
    SplitC<P, KW> fk[NKT];
#pragma unroll
    for (int t = 0; t < NKT; ++t)
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            const int kr = KS == 32 ? kperm32(g, j) : 4 * g + j;
            fk[t].set(j, a.fk[kr * KS + 16 * t + c]);
        }

    // stage-A operands of one block in registers (each wave owns TPW column tiles),
    // with the input-side taps.  The next block's are fetched before and after the B
    // stages (EARLY tiles before), so that they are in flight during the B stages and the
    // write-out (all of them held across the B stages would spill the 32-point stages)
    constexpr int TPW = NT / (ST / 64);
    static_assert(NT % (ST / 64) == 0, "stage-A tiles must divide among the waves");
    c32 xin[TPW][4];
    float tin[SIDE == SIDE_IN ? TPW : 1][SIDE == SIDE_IN ? 4 : 1];
    // every call overwrites all of xin / tin (zeros past the batch), so that they
    // are dead between stage A and the next fetch
    // buffer resources over exactly the block's N points: rows r >= M (n >= N) and blocks past
    // the batch (range 0) read as zero
    auto fetch_range = [&](int64_t bb, auto i0c, auto i1c) {
        constexpr int I0 = decltype(i0c)::value, I1 = decltype(i1c)::value;
        const bool valid = bb < a.nblocks;
        const int64_t bc = valid ? bb : 0;
        const rsrc_t ri = make_rsrc(a.in + bc * N, valid ? uint32_t(N) * 8u : 0u);
        const rsrc_t rt = make_rsrc(a.taps + bc * a.tap_stride, valid ? uint32_t(N) * 4u : 0u);
#pragma unroll
        for (int i = I0; i < I1; ++i) {
            const uint32_t n0 = 16 * (w + i * (ST / 64)) + c + K * 4 * g;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                xin[i][j] = ld_c(ri, n0 * 8u, uint32_t(K * j) * 8u);
                if constexpr (SIDE == SIDE_IN) tin[i][j] = ld_f(rt, n0 * 4u, uint32_t(K * j) * 4u);
            }
        }
    };
    // tiles of the next block requested before the B stages (the rest after them): as many as
    // fit beside the B stages' registers without spilling (measured: BF16 at K = 1024 gains
    // 2-3 % with two, FP16 spills with any)
    constexpr int EARLY = KS == 16 ? TPW : (P::scaled ? 0 : 2);
    auto fetch = [&](int64_t bb) {
        fetch_range(bb, std::integral_constant<int, 0>{}, std::integral_constant<int, TPW>{});
    };


    fetch(blockIdx.x);
    for (int64_t b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
        const rsrc_t rso = make_rsrc(a.out + b * N, uint32_t(N) * 8u);
        const rsrc_t rst = make_rsrc(a.taps + b * a.tap_stride, uint32_t(N) * 4u);

        // ---- stage A: per 16-column tile of p, U = F_M Z, then the coset twiddle
        float sZ = 1.0f;
        if constexpr (P::scaled) {
            float mx = 0.0f;
#pragma unroll
            for (int i = 0; i < TPW; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float f = SIDE == SIDE_IN ? fabsf(tin[i][j]) : 1.0f;
                    mx = fmaxf(mx, fmaxf(fabsf(xin[i][j].x), fabsf(xin[i][j].y)) * f);
                }
            mx = wave_max(mx);
            __syncthreads();
            if (lane == 0) red[w] = mx;
            __syncthreads();
            mx = 0.0f;
#pragma unroll
            for (int q = 0; q < ST / 64; ++q) mx = fmaxf(mx, red[q]);
            sZ = pow2_scale(mx);
        }
        float umax = 0.0f;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int t = w + i * (ST / 64);
            SplitC<P, 4> z;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c32 x = xin[i][j];
                if (conj_io) x = conj(x);
                if constexpr (SIDE == SIDE_IN) x = scale(x, tin[i][j]);
                z.set(j, scale(x, sZ));
            }
            f4 dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
            cmma<P, 4, false>(fm, z, dr, di);
            const int p = 16 * t + c;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 4 * g + j;
                const c32 u = cmul(c32{dr[j], di[j]}, a.ta[p * 16 + m]);
                U[m * RS + p] = u;
                if (m < M) umax = fmaxf(umax, fmaxf(fabsf(u.x), fabsf(u.y)));
            }
        }
        __syncthreads();
        float sU = 1.0f;
        if constexpr (P::scaled) {
            umax = wave_max(umax);
            if (lane == 0) red[w] = umax;
            __syncthreads();
            float mx = 0.0f;
#pragma unroll
            for (int q = 0; q < ST / 64; ++q) mx = fmaxf(mx, red[q]);
            sU = pow2_scale(mx);
        }

        if constexpr (EARLY > 0)
            fetch_range(b + gridDim.x, std::integral_constant<int, 0>{}, std::integral_constant<int, EARLY>{});
        // ---- stages B1, B2: one row m per wave
        for (int m = w; m < M; m += ST / 64) {
            f4 vr[NKT][NKT], vi[NKT][NKT];
#pragma unroll
            for (int tp1 = 0; tp1 < NKT; ++tp1) {
                SplitC<P, KW> A;
#pragma unroll
                for (int j = 0; j < KW; ++j) {
                    const int p2 = KS == 32 ? kperm32(g, j) : 4 * g + j;
                    A.set(j, scale(U[m * RS + 16 * tp1 + c + KS * p2], sU));
                }
#pragma unroll
                for (int tq2 = 0; tq2 < NKT; ++tq2) {
                    vr[tp1][tq2] = f4{0.f, 0.f, 0.f, 0.f};
                    vi[tp1][tq2] = f4{0.f, 0.f, 0.f, 0.f};
                    cmma<P, KW, false>(A, fk[tq2], vr[tp1][tq2], vi[tp1][tq2]);
                }
            }
            // twiddle e^{+j 2 pi p1 q2 / K}; lane holds p1 = 16 tp1 + 4g + j, q2 = 16 tq2 + c
            float vmax = 0.0f;
#pragma unroll
            for (int tp1 = 0; tp1 < NKT; ++tp1)
#pragma unroll
                for (int tq2 = 0; tq2 < NKT; ++tq2)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int p1 = 16 * tp1 + 4 * g + j, q2 = 16 * tq2 + c;
                        const c32 v = cmul(c32{vr[tp1][tq2][j], vi[tp1][tq2][j]}, a.tb[p1 * KS + q2]);
                        vr[tp1][tq2][j] = v.x;
                        vi[tp1][tq2][j] = v.y;
                        vmax = fmaxf(vmax, fmaxf(fabsf(v.x), fabsf(v.y)));
                    }
            float sV = 1.0f;
            if constexpr (P::scaled) sV = pow2_scale(wave_max(vmax));
            // B2: X = F_KS V; the B operand of column tile tq2 is V's D registers
            const float unscale = 1.0f / (sZ * sU * sV);
#pragma unroll
            for (int tq2 = 0; tq2 < NKT; ++tq2) {
                SplitC<P, KW> B;
#pragma unroll
                for (int j = 0; j < KW; ++j) {
                    const int tp1 = j / 4, jj = j % 4;
                    B.set(j, scale(c32{vr[tp1][tq2][jj], vi[tp1][tq2][jj]}, sV));
                }
#pragma unroll
                for (int tq1 = 0; tq1 < NKT; ++tq1) {
                    f4 xr = {0.f, 0.f, 0.f, 0.f}, xi = {0.f, 0.f, 0.f, 0.f};
                    cmma<P, KW, true>(fk[tq1], B, xr, xi);   // F_KS is symmetric: A layout of tile tq1
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int q1 = 16 * tq1 + 4 * g + j, q2 = 16 * tq2 + c;
                        U[m * RS + q2 + KS * q1] = scale(c32{xr[j], xi[j]}, unscale);
                    }
                }
            }
        }
        __syncthreads();
        fetch_range(b + gridDim.x, std::integral_constant<int, EARLY>{}, std::integral_constant<int, TPW>{});

        // ---- natural-order write-out: y_u with u = M q + m; (q, m) advance by ST
        //      per step without a division
        const int dq = ST / M, dm = ST - dq * M;
        int q = int(threadIdx.x) / M, m = int(threadIdx.x) - q * M;
        // eight outputs per thread per step, their output-side taps loaded together
        for (int u0 = threadIdx.x; u0 < N; u0 += 8 * ST) {
            float tv[8];
            if constexpr (SIDE == SIDE_OUT) {
#pragma unroll
                for (int k = 0; k < 8; ++k) tv[k] = ld_f(rst, uint32_t(u0) * 4u, uint32_t(k * ST) * 4u);
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int u = u0 + k * ST;
                if (u < N) {
                    c32 y = U[m * RS + q];
                    if (conj_io) y = conj(y);
                    if constexpr (SIDE == SIDE_OUT) y = scale(y, tv[k]);
                    st_c(y, rso, uint32_t(u) * 8u, 0u);
                }
                q += dq;
                m += dm;
                if (m >= M) {
                    m -= M;
                    ++q;
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side
struct SplitTables {
    c32 *fm = nullptr, *fk = nullptr, *ta = nullptr, *tb = nullptr;
};

static std::mutex g_split_mu;
static std::map<std::tuple<int, int, int>, SplitTables> g_split_tables;   // (device, K, M)

static c32 root(long k, long n)
{
    k %= n;
    const double ang = 2.0 * M_PI * double(k) / double(n);
    return c32{float(std::cos(ang)), float(std::sin(ang))};
}

static int upload_table(const std::vector<c32> &h, c32 **d)
{
    hipError_t e = hipMalloc(d, h.size() * sizeof(c32));
    if (e != hipSuccess) {
        set_error("hipMalloc(split table)", e);
        return TF_EHIP;
    }
    e = hipMemcpy(*d, h.data(), h.size() * sizeof(c32), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error("hipMemcpy(split table)", e);
        return TF_EHIP;
    }
    return TF_OK;
}

static int split_tables(int K, int M, SplitTables **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return TF_EHIP;
    std::lock_guard<std::mutex> lk(g_split_mu);
    auto it = g_split_tables.find({dev, K, M});
    if (it == g_split_tables.end()) {
        const int KS = K == 1024 ? 32 : 16;
        const long N = long(K) * M;
        std::vector<c32> fm(256, c32{0.f, 0.f}), fk(KS * KS), ta(size_t(K) * 16), tb(KS * KS);
        for (int m = 0; m < M; ++m)
            for (int r = 0; r < M; ++r) fm[m * 16 + r] = root(long(m) * r, M);
        for (int x = 0; x < KS; ++x)
            for (int y = 0; y < KS; ++y) {
                fk[x * KS + y] = root(long(x) * y, KS);
                tb[x * KS + y] = root(long(x) * y, K);
            }
        for (int p = 0; p < K; ++p)
            for (int m = 0; m < 16; ++m) ta[p * 16 + m] = root(long(p) * m, N);
        SplitTables t;
        int rc = upload_table(fm, &t.fm);
        if (!rc) rc = upload_table(fk, &t.fk);
        if (!rc) rc = upload_table(ta, &t.ta);
        if (!rc) rc = upload_table(tb, &t.tb);
        if (rc) return rc;
        it = g_split_tables.emplace(std::make_tuple(dev, K, M), t).first;
    }
    *out = &it->second;
    return TF_OK;
}

int split_supported(int K, int M, int compute)
{
    if (compute != TF_SPLIT_BF16 && compute != TF_SPLIT_FP16) return TF_EUNSUPPORTED;
    if ((K != 256 && K != 1024) || M < 1 || M > 16) return TF_EUNSUPPORTED;
    return TF_OK;
}

size_t split_workspace_size(int64_t, int, int, int64_t, int, int) { return 0; }

int split_prepare(int K, int M, int compute)
{
    int rc = split_supported(K, M, compute);
    if (rc) return rc;
    SplitTables *t = nullptr;
    return split_tables(K, M, &t);
}

template <int KS, class P>
static hipError_t launch_split(int side, const SplitArgs &a, unsigned grid, hipStream_t s)
{
    if (side == SIDE_IN)
        hipLaunchKernelGGL((split_kernel<KS, P, SIDE_IN>), dim3(grid), dim3(ST), 0, s, a);
    else
        hipLaunchKernelGGL((split_kernel<KS, P, SIDE_OUT>), dim3(grid), dim3(ST), 0, s, a);
    return hipGetLastError();
}

int split_run(int direction, const void *in, const float *taps, void *out, int64_t nblocks, int K, int M,
              int64_t tap_stride, int compute, void *, size_t, void *stream)
{
    int rc = split_supported(K, M, compute);
    if (rc) return rc;
    SplitTables *t = nullptr;
    rc = split_tables(K, M, &t);
    if (rc) return rc;
    SplitArgs a{};
    a.in = reinterpret_cast<const c32 *>(in);
    a.out = reinterpret_cast<c32 *>(out);
    a.taps = taps;
    a.fm = t->fm;
    a.fk = t->fk;
    a.ta = t->ta;
    a.tb = t->tb;
    a.nblocks = nblocks;
    a.tap_stride = tap_stride;
    a.M = M;
    // persistent grid: about two resident rounds of workgroups, so that each
    // workgroup prefetches its next block while it finishes the current one
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int per_cu = K == 1024 ? 1 : 2;
    const unsigned grid = unsigned(std::min<int64_t>(nblocks, int64_t(cus) * per_cu));
    const int side = direction == 0 ? SIDE_IN : SIDE_OUT;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    if (K == 1024)
        e = compute == TF_SPLIT_BF16 ? launch_split<32, PrecBF16>(side, a, grid, s)
                                     : launch_split<32, PrecFP16>(side, a, grid, s);
    else
        e = compute == TF_SPLIT_BF16 ? launch_split<16, PrecBF16>(side, a, grid, s)
                                     : launch_split<16, PrecFP16>(side, a, grid, s);
    if (e != hipSuccess) {
        set_error("split launch", e);
        return TF_EHIP;
    }
    return TF_OK;
}

} // namespace bt
