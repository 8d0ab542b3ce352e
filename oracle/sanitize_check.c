/*
 * Sanitizer driver for the FP64 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Built by tests/test_sanitizers.py together with oracle.c under gcc's
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only), and run
 * on the CPU.  Every array is allocated at its exact size, so a read or write
 * past any block, tap or output region aborts the run.  It exercises each
 * entry point of oracle.c on a ragged batch of block sizes 1..48 laid out
 * with gaps and in shuffled order, and checks relations that hold whatever
 * the layout: the inverse undoes the forward, and <T S, y> = <S, T^H y> for
 * the forward / adjoint and the decimated pair.  Exit status 0 means no
 * sanitizer report and every relation within 1e-10.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_forward(int64_t, const int64_t *, const int64_t *, const int64_t *, const double *,
                   const double *, double *, int);
int oracle_inverse(int64_t, const int64_t *, const int64_t *, const int64_t *, const double *,
                   const double *, double *, int64_t *, int);
int oracle_adjoint(int64_t, const int64_t *, const int64_t *, const int64_t *, const double *,
                   const double *, const double *, double *, double *, int);
int oracle_inverse_adjoint(int64_t, const int64_t *, const int64_t *, const int64_t *, const double *,
                           const double *, const double *, double *, double *, int);
int oracle_decimated(int64_t, const int64_t *, const int64_t *, const int64_t *, const int64_t *,
                     const int64_t *, const double *, const double *, double *, int);
int oracle_decimated_adjoint(int64_t, const int64_t *, const int64_t *, const int64_t *,
                             const int64_t *, const int64_t *, const double *, const double *,
                             double *, int);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double urand(void) /* xorshift64*, uniform in [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
}

static double *alloc_d(size_t n)
{
    double *p = (double *)malloc(sizeof(double) * (n ? n : 1));
    if (!p) exit(3);
    return p;
}

/* Re <a, b> over the blocks' regions of two interleaved complex arrays */
static double dot_re(int64_t nb, const int64_t *N, const int64_t *off, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < nb; ++i)
        for (int64_t n = 0; n < N[i]; ++n) {
            const double *x = a + 2 * (off[i] + n), *y = b + 2 * (off[i] + n);
            s += x[0] * y[0] + x[1] * y[1];
        }
    return s;
}

int main(void)
{
    enum { NB = 48 };
    int64_t N[NB], K[NB], x_off[NB], tap_off[NB], y_off[NB];
    int64_t order[NB];
    for (int64_t i = 0; i < NB; ++i) order[i] = i;
    for (int64_t i = NB - 1; i > 0; --i) { /* shuffled memory order */
        int64_t j = (int64_t)(urand() * (double)(i + 1));
        int64_t t = order[i]; order[i] = order[j]; order[j] = t;
    }
    int64_t pos = 0, tpos = 0, ypos = 0;
    for (int64_t k = 0; k < NB; ++k) {
        int64_t i = order[k];
        N[i] = i + 1;
        /* decimation factor: the largest of 1, 2, 3, 4 that divides N */
        K[i] = N[i];
        for (int64_t m = 4; m >= 2; --m)
            if (N[i] % m == 0) { K[i] = N[i] / m; break; }
        pos += (k % 3);                      /* gaps between blocks */
        x_off[i] = pos; pos += N[i];
        tap_off[i] = tpos; tpos += N[i];
        y_off[i] = ypos; ypos += K[i];
    }
    const size_t total = (size_t)pos, ttotal = (size_t)tpos, ytotal = (size_t)ypos;
    double *S = alloc_d(2 * total), *y = alloc_d(2 * total), *S2 = alloc_d(2 * total);
    double *yb = alloc_d(2 * total), *Sb = alloc_d(2 * total), *tb = alloc_d(total);
    double *g = alloc_d(2 * total), *taps = alloc_d(ttotal);
    double *d = alloc_d(2 * ytotal), *db = alloc_d(2 * ytotal), *Sd = alloc_d(2 * total);
    for (size_t i = 0; i < 2 * total; ++i) { S[i] = urand() - 0.5; yb[i] = urand() - 0.5; g[i] = 0.0; Sb[i] = 0.0; Sd[i] = 0.0; y[i] = 0.0; S2[i] = 0.0; }
    for (size_t i = 0; i < total; ++i) tb[i] = 0.0;
    for (size_t i = 0; i < ttotal; ++i) taps[i] = 0.5 + urand();
    for (size_t i = 0; i < 2 * ytotal; ++i) db[i] = urand() - 0.5;
    int64_t nz = -1;
    int bad = 0;
    for (int threads = 1; threads <= 2; ++threads) {
        bad |= oracle_forward(NB, N, x_off, tap_off, S, taps, y, threads);
        bad |= oracle_inverse(NB, N, x_off, tap_off, y, taps, S2, &nz, threads);
        bad |= oracle_adjoint(NB, N, x_off, tap_off, yb, taps, S, Sb, tb, threads);
        bad |= oracle_inverse_adjoint(NB, N, x_off, tap_off, yb, taps, S2, g, tb, threads);
        bad |= oracle_decimated(NB, N, K, x_off, tap_off, y_off, S, taps, d, threads);
        bad |= oracle_decimated_adjoint(NB, N, K, x_off, tap_off, y_off, db, taps, Sd, threads);
    }
    if (bad || nz != 0) { fprintf(stderr, "oracle call failed\n"); return 1; }
    double err = 0.0, ref = 0.0;
    for (int64_t i = 0; i < NB; ++i)
        for (int64_t n = 0; n < 2 * N[i]; ++n) {
            const double e = S2[2 * x_off[i] + n] - S[2 * x_off[i] + n];
            err += e * e;
            ref += S[2 * x_off[i] + n] * S[2 * x_off[i] + n];
        }
    const double rt = sqrt(err / ref);
    const double lhs = dot_re(NB, N, x_off, y, yb), rhs = dot_re(NB, N, x_off, S, Sb);
    /* decimated pair: <D S, db> over the K-point outputs equals <S, D^H db> */
    double dl = 0.0;
    for (int64_t i = 0; i < NB; ++i)
        for (int64_t q = 0; q < K[i]; ++q) {
            const double *a = d + 2 * (y_off[i] + q), *b = db + 2 * (y_off[i] + q);
            dl += a[0] * b[0] + a[1] * b[1];
        }
    const double dr = dot_re(NB, N, x_off, S, Sd);
    printf("round trip %.3e  adjoint %.3e  decimated adjoint %.3e\n", rt, fabs(lhs - rhs) / fabs(rhs),
           fabs(dl - dr) / fabs(dr));
    free(S); free(y); free(S2); free(yb); free(Sb); free(tb); free(g); free(taps); free(d); free(db); free(Sd);
    return (rt < 1e-10 && fabs(lhs - rhs) <= 1e-10 * fabs(rhs) && fabs(dl - dr) <= 1e-10 * fabs(dr)) ? 0 : 2;
}
