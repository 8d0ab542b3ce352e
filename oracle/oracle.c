/*
 * FP64 CPU oracle for the block transform -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the package's smoke check and the benchmark's CPU
 * baseline call this code.  It shares nothing with the GPU library: no
 * headers, no tables, no helpers.
 *
 * What is computed (J. Selva, "Non-iterative type 4 and 5 nonuniform FFT
 * methods in the one-dimensional case"):
 *
 *   The regular-grid step of the method evaluates a filtered trigonometric
 *   polynomial  gamma(t) = sum_{n<N} Lambda_n S_n e^{j 2 pi n t}  (eq. (6),
 *   with the kernel coefficients Lambda of eq. (4)) on the uniform grid
 *   t = u/N.  With omega^k = exp(+j 2 pi (k mod N)/N), per block:
 *
 *     forward          y_u  = sum_n Lambda_n S_n omega^{n u}                 (eq. (6); eq. (7) is u = M q)
 *     inverse          S_n  = (N Lambda_n)^{-1} sum_u y_u omega^{-n u}      (eq. (31), with the
 *                                                                            damping filter of eq. (8)
 *                                                                            generalised to any
 *                                                                            nonzero real filter)
 *     adjoint          W_n  = sum_u ybar_u omega^{-n u}
 *                      Sbar_n = Lambda_n W_n,  Lambdabar_n = Re(conj(S_n) W_n)
 *                      (the Hermitian of the forward matrix; the type-4/type-5
 *                      duality of Sec. 6 is the same statement for the NUDFT)
 *     inverse adjoint  ybar_u = sum_n omega^{+n u} gbar_n / (N Lambda_n)
 *                      Lambdabar_n = -Re(conj(gbar_n) S_n) / Lambda_n
 *     decimated        gamma(q/K) = sum_n Lambda_n S_n e^{j 2 pi n q / K}, q < K   (eq. (7): the
 *                      polynomial of eq. (6) with R = eta P coefficients, read at P
 *                      regular points; here P = K and eta = M)
 *     decimated adj.   Sbar_n = Lambda_n sum_q ybar_q e^{-j 2 pi n q / K}
 *
 *   DFT sign and normalisation follow eq. (0) (negative exponent, no 1/P);
 *   the IDFT carries 1/P, which is what makes eq. (7) read P * IDFT{...}.
 *
 * Every sum is the plain O(N^2) definition, in double precision, with the
 * exponent n*u reduced modulo N as an integer before the angle is formed.
 * Complex numbers are interleaved (re, im) doubles.  Blocks are independent
 * and are spread over OpenMP threads; nothing inside a block is reordered.
 *
 * Ragged batches: block b has N[b] points starting at complex offset x_off[b]
 * and N[b] taps starting at tap_off[b] (all offsets in elements).  Per-block
 * tap gradients are written at x_off[b] (summing them over blocks that share
 * taps is left to the caller).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_TWO_PI 6.283185307179586476925286766559

/* cos/sin of 2 pi k / N for k < N */
static int roots_of_unity(int64_t N, double **c_out, double **s_out)
{
    double *c = (double *)malloc(sizeof(double) * (size_t)N);
    double *s = (double *)malloc(sizeof(double) * (size_t)N);
    if (!c || !s) { free(c); free(s); return -1; }
    for (int64_t k = 0; k < N; ++k) {
        double ang = ORACLE_TWO_PI * (double)k / (double)N;
        c[k] = cos(ang);
        s[k] = sin(ang);
    }
    *c_out = c;
    *s_out = s;
    return 0;
}

/*
 * out_v = sum_w in_w * exp(sign * j 2 pi (v*w mod L) / L)  for v < Lout, w < Lin,
 * with L the period of the exponential.  in may be scaled per element by
 * scale_in (NULL = 1).  This is the one plain matrix-vector definition every
 * entry point below is written in.
 */
static void dft_sum(int64_t L, int64_t Lin, int64_t Lout, int sign,
                    const double *c, const double *s,
                    const double *in_re, const double *in_im, double *out)
{
    for (int64_t v = 0; v < Lout; ++v) {
        double acc_re = 0.0, acc_im = 0.0;
        int64_t step = v % L;
        int64_t k = 0;                          /* (v * w) mod L */
        for (int64_t w = 0; w < Lin; ++w) {
            double wr = c[k];
            double wi = sign > 0 ? s[k] : -s[k];
            acc_re += in_re[w] * wr - in_im[w] * wi;
            acc_im += in_re[w] * wi + in_im[w] * wr;
            k += step;
            if (k >= L) k -= L;
        }
        out[2 * v] = acc_re;
        out[2 * v + 1] = acc_im;
    }
}

#ifdef _OPENMP
#define ORACLE_SET_THREADS(nt) do { if ((nt) > 0) omp_set_num_threads(nt); } while (0)
#else
#define ORACLE_SET_THREADS(nt) do { (void)(nt); } while (0)
#endif

/* forward: y_u = sum_n Lambda_n S_n omega^{nu} */
int oracle_forward(int64_t nblocks, const int64_t *N, const int64_t *x_off, const int64_t *tap_off,
                   const double *S, const double *taps, double *y, int nthreads)
{
    int err = 0;
    ORACLE_SET_THREADS(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t n_b = N[b];
        double *c = NULL, *s = NULL;
        double *zr = (double *)malloc(sizeof(double) * (size_t)n_b);
        double *zi = (double *)malloc(sizeof(double) * (size_t)n_b);
        if (!zr || !zi || roots_of_unity(n_b, &c, &s)) { err |= 1; free(zr); free(zi); continue; }
        const double *Sb = S + 2 * x_off[b];
        const double *Lb = taps + tap_off[b];
        for (int64_t n = 0; n < n_b; ++n) {     /* the filter multiply of eq. (6) */
            zr[n] = Lb[n] * Sb[2 * n];
            zi[n] = Lb[n] * Sb[2 * n + 1];
        }
        dft_sum(n_b, n_b, n_b, +1, c, s, zr, zi, y + 2 * x_off[b]);
        free(zr); free(zi); free(c); free(s);
    }
    return err ? -1 : 0;
}

/* inverse: S_n = (N Lambda_n)^{-1} sum_u y_u omega^{-nu}; counts zero taps */
int oracle_inverse(int64_t nblocks, const int64_t *N, const int64_t *x_off, const int64_t *tap_off,
                   const double *y, const double *taps, double *S, int64_t *nzero, int nthreads)
{
    int err = 0;
    int64_t zeros = 0;
    ORACLE_SET_THREADS(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err) reduction(+ : zeros)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t n_b = N[b];
        double *c = NULL, *s = NULL;
        double *yr = (double *)malloc(sizeof(double) * (size_t)n_b);
        double *yi = (double *)malloc(sizeof(double) * (size_t)n_b);
        if (!yr || !yi || roots_of_unity(n_b, &c, &s)) { err |= 1; free(yr); free(yi); continue; }
        const double *yb = y + 2 * x_off[b];
        for (int64_t u = 0; u < n_b; ++u) { yr[u] = yb[2 * u]; yi[u] = yb[2 * u + 1]; }
        double *Sb = S + 2 * x_off[b];
        dft_sum(n_b, n_b, n_b, -1, c, s, yr, yi, Sb);
        const double *Lb = taps + tap_off[b];
        for (int64_t n = 0; n < n_b; ++n) {     /* the 1/(N Lambda_n) of eq. (31) */
            if (Lb[n] == 0.0) zeros += 1;
            double d = (double)n_b * Lb[n];
            Sb[2 * n] = Sb[2 * n] / d;
            Sb[2 * n + 1] = Sb[2 * n + 1] / d;
        }
        free(yr); free(yi); free(c); free(s);
    }
    if (nzero) *nzero = zeros;
    return err ? -1 : 0;
}

/* adjoint of the forward: Sbar = Lambda (.) W, Lambdabar = Re(conj(S) (.) W), W = DFT(ybar) */
int oracle_adjoint(int64_t nblocks, const int64_t *N, const int64_t *x_off, const int64_t *tap_off,
                   const double *ybar, const double *taps, const double *S,
                   double *Sbar, double *tapbar, int nthreads)
{
    int err = 0;
    ORACLE_SET_THREADS(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t n_b = N[b];
        double *c = NULL, *s = NULL;
        double *yr = (double *)malloc(sizeof(double) * (size_t)n_b);
        double *yi = (double *)malloc(sizeof(double) * (size_t)n_b);
        double *W = (double *)malloc(sizeof(double) * 2 * (size_t)n_b);
        if (!yr || !yi || !W || roots_of_unity(n_b, &c, &s)) {
            err |= 1; free(yr); free(yi); free(W); continue;
        }
        const double *yb = ybar + 2 * x_off[b];
        for (int64_t u = 0; u < n_b; ++u) { yr[u] = yb[2 * u]; yi[u] = yb[2 * u + 1]; }
        dft_sum(n_b, n_b, n_b, -1, c, s, yr, yi, W);
        const double *Lb = taps + tap_off[b];
        for (int64_t n = 0; n < n_b; ++n) {
            if (Sbar) {
                Sbar[2 * (x_off[b] + n)] = Lb[n] * W[2 * n];
                Sbar[2 * (x_off[b] + n) + 1] = Lb[n] * W[2 * n + 1];
            }
            if (tapbar && S) {
                const double *Sn = S + 2 * (x_off[b] + n);
                tapbar[x_off[b] + n] = Sn[0] * W[2 * n] + Sn[1] * W[2 * n + 1];
            }
        }
        free(yr); free(yi); free(W); free(c); free(s);
    }
    return err ? -1 : 0;
}

/* adjoint of the inverse: ybar_u = sum_n omega^{nu} gbar_n/(N Lambda_n);
   Lambdabar_n = -Re(conj(gbar_n) Shat_n)/Lambda_n */
int oracle_inverse_adjoint(int64_t nblocks, const int64_t *N, const int64_t *x_off, const int64_t *tap_off,
                           const double *gbar, const double *taps, const double *Shat,
                           double *ybar, double *tapbar, int nthreads)
{
    int err = 0;
    ORACLE_SET_THREADS(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t n_b = N[b];
        double *c = NULL, *s = NULL;
        double *zr = (double *)malloc(sizeof(double) * (size_t)n_b);
        double *zi = (double *)malloc(sizeof(double) * (size_t)n_b);
        if (!zr || !zi || roots_of_unity(n_b, &c, &s)) { err |= 1; free(zr); free(zi); continue; }
        const double *gb = gbar + 2 * x_off[b];
        const double *Lb = taps + tap_off[b];
        for (int64_t n = 0; n < n_b; ++n) {
            double d = (double)n_b * Lb[n];
            zr[n] = gb[2 * n] / d;
            zi[n] = gb[2 * n + 1] / d;
            if (tapbar && Shat) {
                const double *Sn = Shat + 2 * (x_off[b] + n);
                tapbar[x_off[b] + n] = -(gb[2 * n] * Sn[0] + gb[2 * n + 1] * Sn[1]) / Lb[n];
            }
        }
        if (ybar) dft_sum(n_b, n_b, n_b, +1, c, s, zr, zi, ybar + 2 * x_off[b]);
        free(zr); free(zi); free(c); free(s);
    }
    return err ? -1 : 0;
}

/* decimated forward, eq. (7): out_q = sum_n Lambda_n S_n e^{j 2 pi n q / K}, q < K.
   Block b reads N[b] = K[b] * M[b] coefficients at x_off[b] and writes K[b] values
   at y_off[b]. */
int oracle_decimated(int64_t nblocks, const int64_t *N, const int64_t *K,
                     const int64_t *x_off, const int64_t *tap_off, const int64_t *y_off,
                     const double *S, const double *taps, double *out, int nthreads)
{
    int err = 0;
    ORACLE_SET_THREADS(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t n_b = N[b], k_b = K[b];
        double *c = NULL, *s = NULL;
        double *zr = (double *)malloc(sizeof(double) * (size_t)n_b);
        double *zi = (double *)malloc(sizeof(double) * (size_t)n_b);
        if (!zr || !zi || roots_of_unity(k_b, &c, &s)) { err |= 1; free(zr); free(zi); continue; }
        const double *Sb = S + 2 * x_off[b];
        const double *Lb = taps + tap_off[b];
        for (int64_t n = 0; n < n_b; ++n) {
            zr[n] = Lb[n] * Sb[2 * n];
            zi[n] = Lb[n] * Sb[2 * n + 1];
        }
        dft_sum(k_b, n_b, k_b, +1, c, s, zr, zi, out + 2 * y_off[b]);
        free(zr); free(zi); free(c); free(s);
    }
    return err ? -1 : 0;
}

/* adjoint of the decimated forward: Sbar_n = Lambda_n sum_q ybar_q e^{-j 2 pi n q / K} */
int oracle_decimated_adjoint(int64_t nblocks, const int64_t *N, const int64_t *K,
                             const int64_t *x_off, const int64_t *tap_off, const int64_t *y_off,
                             const double *ybar, const double *taps, double *Sbar, int nthreads)
{
    int err = 0;
    ORACLE_SET_THREADS(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t b = 0; b < nblocks; ++b) {
        int64_t n_b = N[b], k_b = K[b];
        double *c = NULL, *s = NULL;
        double *yr = (double *)malloc(sizeof(double) * (size_t)k_b);
        double *yi = (double *)malloc(sizeof(double) * (size_t)k_b);
        if (!yr || !yi || roots_of_unity(k_b, &c, &s)) { err |= 1; free(yr); free(yi); continue; }
        const double *yb = ybar + 2 * y_off[b];
        for (int64_t q = 0; q < k_b; ++q) { yr[q] = yb[2 * q]; yi[q] = yb[2 * q + 1]; }
        double *Sb = Sbar + 2 * x_off[b];
        dft_sum(k_b, k_b, n_b, -1, c, s, yr, yi, Sb);
        const double *Lb = taps + tap_off[b];
        for (int64_t n = 0; n < n_b; ++n) {
            Sb[2 * n] *= Lb[n];
            Sb[2 * n + 1] *= Lb[n];
        }
        free(yr); free(yi); free(c); free(s);
    }
    return err ? -1 : 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
