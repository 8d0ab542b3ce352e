// Unfused comparison path ("plain FP32"): the four stages of the transform as
// separate kernels with HBM round trips between them and no LDS staging.
//
// Forward, with n = p + K r and u = M q + m (the staging behind eq. (7)):
//   stage i   Z_n = Lambda_n S_n                                 (filter multiply)
//   stage ii  U[m][p] = sum_{r<M} Z_{p+Kr} e^{+j 2 pi r m / M}   (circular fold, all cosets)
//   stage iii U[m][p] *= e^{+j 2 pi p m / N}                     (coset twiddle)
//   stage iv  y_{Mq+m} = sum_{p<K} U[m][p] e^{+j 2 pi p q / K}   (length-K IDFT, radix-2
//                                                                 Stockham passes in HBM)
// The negative-exponent directions conjugate on the way in and out.  Twiddles
// come from one table of the N-th roots of unity per (K, M).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bt_dft.hpp"
#include "bt_plain.hpp"

namespace bt {

// stage i: z = op(in); op = conj?, times Lambda or 1/(N Lambda)
__global__ void plain_in_kernel(PlainArgs a, const c32 *in, c32 *z)
{
    const int64_t N = int64_t(a.K) * a.M;
    const int64_t total = a.nblocks * N;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = i / N, n = i - b * N;
        c32 x = in[i];
        if (a.conj_io) x = conj(x);
        const float *tp = a.taps + b * a.tap_stride;
        if (a.in_op == IN_MUL_TAP) x = scale(x, tp[n]);
        else if (a.in_op == IN_DIV_NTAP) x = scale(x, 1.0f / (float(N) * tp[n]));
        z[i] = x;
    }
}

// stage ii: U[b][m][p] = sum_r z[b][p + K r] w_M^{r m}
__global__ void plain_fold_kernel(PlainArgs a, const c32 *z, c32 *U)
{
    const int64_t K = a.K, M = a.M, N = K * M;
    const int64_t total = a.nblocks * N;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = i / N, rem = i - b * N, m = rem / K, p = rem - m * K;
        c32 acc = c32{0.f, 0.f};
        for (int64_t r = 0; r < M; ++r) {
            const c32 w = a.roots[((r * m) % M) * K];      // e^{+j 2 pi r m / M}
            acc = acc + cmul(z[b * N + p + K * r], w);
        }
        U[i] = acc;
    }
}

// stage iii: U[b][m][p] *= w_N^{p m}
__global__ void plain_twiddle_kernel(PlainArgs a, c32 *U)
{
    const int64_t K = a.K, M = a.M, N = K * M;
    const int64_t total = a.nblocks * N;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t rem = i % N, m = rem / K, p = rem - m * K;
        U[i] = cmul(U[i], a.roots[(p * m) % N]);
    }
}

// stage iv, one radix-2 Stockham pass over every row (b, m) of length K:
//   v0 = x[j], v1 = x[j + K/2] w_{2 Ns}^{j mod Ns};  x'[(j/Ns) 2Ns + j mod Ns (+Ns)] = v0 +- v1.
// The last pass writes row (b, m), element q, to y[b][M q + m] after the output op.
__global__ void plain_radix2_kernel(PlainArgs a, const c32 *src, c32 *dst, int Ns, int last,
                                    float *tg_part)
{
    const int64_t K = a.K, M = a.M, N = K * M, H = K / 2;
    const int64_t total = a.nblocks * M * H;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t row = i / H, j = i - row * H;
        const int64_t jm = j % Ns;
        const c32 *x = src + row * K;
        const c32 w = a.roots[jm * (N / (2 * Ns))];          // e^{+j 2 pi jm / (2 Ns)}
        const c32 v0 = x[j], v1 = cmul(x[j + H], w);
        const int64_t o = (j / Ns) * 2 * Ns + jm;
        const c32 s0 = v0 + v1, s1 = v0 - v1;
        if (!last) {
            dst[row * K + o] = s0;
            dst[row * K + o + Ns] = s1;
        } else {
            const int64_t b = row / M, m = row - b * M;
            const float *tp = a.taps + b * a.tap_stride;
            const c32 outs[2] = {s0, s1};
            for (int h = 0; h < 2; ++h) {
                const int64_t q = o + h * Ns;
                const int64_t k = M * q + m;
                c32 w2 = outs[h];
                if (a.conj_io) w2 = conj(w2);
                if (a.tg_op == TG_OUT) {
                    const c32 s = a.aux[b * N + k];
                    tg_part[b * N + k] = s.x * w2.x + s.y * w2.y;
                }
                if (a.out_op == OUT_MUL_TAP) w2 = scale(w2, tp[k]);
                else if (a.out_op == OUT_DIV_NTAP) {
                    if (tp[k] == 0.0f && a.status) *a.status = 1;
                    w2 = scale(w2, 1.0f / (float(N) * tp[k]));
                }
                a.out[b * N + k] = w2;
            }
        }
    }
}

// K = 1: the last stage is the identity on each row; apply the output op.
__global__ void plain_copy_out_kernel(PlainArgs a, const c32 *U, float *tg_part)
{
    const int64_t M = a.M, N = M;
    const int64_t total = a.nblocks * N;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = i / N, k = i - b * N;
        const float *tp = a.taps + b * a.tap_stride;
        c32 w2 = U[i];
        if (a.conj_io) w2 = conj(w2);
        if (a.tg_op == TG_OUT) tg_part[i] = a.aux[i].x * w2.x + a.aux[i].y * w2.y;
        if (a.out_op == OUT_MUL_TAP) w2 = scale(w2, tp[k]);
        else if (a.out_op == OUT_DIV_NTAP) {
            if (tp[k] == 0.0f && a.status) *a.status = 1;
            w2 = scale(w2, 1.0f / (float(N) * tp[k]));
        }
        a.out[i] = w2;
    }
}

// tap gradient rows -> partial sums: part2[c][k] = sum_{r in chunk c} part[r][k]; the
// chunks are strided over gridDim.y (at most 65535), so any row count is covered
__global__ void rows_reduce_kernel(const float *part, int64_t rows, int64_t n, int64_t chunk,
                                   float *out)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k >= n) return;
    const int64_t nch = (rows + chunk - 1) / chunk;
    for (int64_t c = blockIdx.y; c < nch; c += gridDim.y) {
        const int64_t r0 = c * chunk;
        const int64_t r1 = (r0 + chunk < rows) ? r0 + chunk : rows;
        float acc = 0.0f;
#pragma unroll 8
        for (int64_t r = r0; r < r1; ++r) acc += part[r * n + k];   // loads issued ahead, adds in row order
        out[c * n + k] = acc;
    }
}

static unsigned grid_for(int64_t work, int threads)
{
    int64_t g = (work + threads - 1) / threads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return unsigned(g);
}

hipError_t plain_run(const PlainArgs &a, const c32 *in, c32 *ws0, c32 *ws1, float *tg_part,
                     hipStream_t s)
{
    const int64_t N = int64_t(a.K) * a.M;
    const int64_t total = a.nblocks * N;
    const int T = 256;
    hipLaunchKernelGGL(plain_in_kernel, dim3(grid_for(total, T)), dim3(T), 0, s, a, in, ws0);
    hipLaunchKernelGGL(plain_fold_kernel, dim3(grid_for(total, T)), dim3(T), 0, s, a, ws0, ws1);
    hipLaunchKernelGGL(plain_twiddle_kernel, dim3(grid_for(total, T)), dim3(T), 0, s, a, ws1);
    if (a.K == 1) {
        hipLaunchKernelGGL(plain_copy_out_kernel, dim3(grid_for(total, T)), dim3(T), 0, s, a, ws1,
                           tg_part);
        return hipGetLastError();
    }
    const c32 *src = ws1;
    c32 *dst = ws0;
    for (int Ns = 1; Ns < a.K; Ns *= 2) {
        const int last = (2 * Ns == a.K);
        hipLaunchKernelGGL(plain_radix2_kernel, dim3(grid_for(total / 2, T)), dim3(T), 0, s, a, src,
                           dst, Ns, last, tg_part);
        const c32 *t = dst;
        dst = const_cast<c32 *>(src);
        src = t;
    }
    return hipGetLastError();
}

hipError_t rows_reduce(const float *part, int64_t rows, int64_t n, float *scratch, float *out,
                       hipStream_t s)
{
    // two fixed-order stages: chunks of ROWS_REDUCE_CHUNK rows (many workgroups, short
    // loops), then the chunk sums
    const int T = 256;
    const int64_t chunk = ROWS_REDUCE_CHUNK;
    const int64_t nch = rows_reduce_chunks(rows);
    if (nch <= 1) {
        hipLaunchKernelGGL(rows_reduce_kernel, dim3(grid_for(n, T), 1), dim3(T), 0, s, part, rows, n,
                           rows > 0 ? rows : 1, out);
        return hipGetLastError();
    }
    const unsigned gy = unsigned(nch < 65535 ? nch : 65535);
    hipLaunchKernelGGL(rows_reduce_kernel, dim3(grid_for(n, T), gy), dim3(T), 0, s, part,
                       rows, n, chunk, scratch);
    hipLaunchKernelGGL(rows_reduce_kernel, dim3(grid_for(n, T), 1), dim3(T), 0, s,
                       (const float *)scratch, nch, n, nch, out);
    return hipGetLastError();
}

} // namespace bt
