// Register-resident short DFTs for the block transform (gfx950).
//
// Every codelet computes, in place, X_k = sum_n v_n exp(+j 2 pi n k / R) for
// k < R -- the positive-exponent transform that the forward evaluation of the
// trigonometric polynomial (eq. (6), grid form eq. (7)) needs.  The negative
// exponent of the DFT in eq. (0) is obtained by conjugating inputs and
// outputs, which is exact.
//
// All indices and twiddle constants are compile-time values once the loops
// below are unrolled, so the permutations cost nothing and the constants are
// folded (computed here in double and rounded once to float).  Trivial
// rotations (1, j, -1, -j and the odd multiples of pi/4) are special-cased.
//
// Radices: powers of two through Cooley-Tukey composition of radix 2/4;
// odd R through the symmetric-pair direct form; coprime products (6, 10, 12,
// 14, 15) through the Good-Thomas prime-factor map (no twiddles).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define BT_HD __host__ __device__ __forceinline__

namespace bt {

struct c32 {
    float x, y;
};

BT_HD c32 mk(float x, float y) { return c32{x, y}; }
BT_HD c32 operator+(c32 a, c32 b) { return c32{a.x + b.x, a.y + b.y}; }
BT_HD c32 operator-(c32 a, c32 b) { return c32{a.x - b.x, a.y - b.y}; }
BT_HD c32 operator-(c32 a) { return c32{-a.x, -a.y}; }
BT_HD c32 cmul(c32 a, c32 b) { return c32{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
BT_HD c32 cmulc(c32 a, c32 b) { return c32{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; } // a * conj(b)
BT_HD c32 conj(c32 a) { return c32{a.x, -a.y}; }
BT_HD c32 mul_j(c32 a) { return c32{-a.y, a.x}; }          // j a
BT_HD c32 scale(c32 a, float s) { return c32{a.x * s, a.y * s}; }

// ------------------------------------------------------------------ compile-time trig
constexpr double kPiOver2 = 1.57079632679489661923132169163975144;

constexpr double ct_sin_poly(double x)   // |x| <= pi/4
{
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 14; ++i) {
        term *= -x2 / double((2 * i) * (2 * i + 1));
        sum += term;
    }
    return sum;
}

constexpr double ct_cos_poly(double x)   // |x| <= pi/4
{
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 14; ++i) {
        term *= -x2 / double((2 * i - 1) * (2 * i));
        sum += term;
    }
    return sum;
}

// cos and sin of 2 pi k / n, octant-reduced with integer arithmetic
constexpr double ct_cos2pi(long k, long n, bool want_sin)
{
    k %= n;
    if (k < 0) k += n;
    long k4 = 4 * k;
    long quad = k4 / n;                 // quadrant 0..3
    long rem = k4 - quad * n;           // angle within the quadrant: (pi/2) rem / n
    bool flip = 2 * rem > n;            // use the complementary angle
    double x = kPiOver2 * double(flip ? (n - rem) : rem) / double(n);
    double c0 = flip ? ct_sin_poly(x) : ct_cos_poly(x);   // cos of the in-quadrant angle
    double s0 = flip ? ct_cos_poly(x) : ct_sin_poly(x);
    double c = 0, s = 0;
    switch (quad) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
    }
    return want_sin ? s : c;
}

constexpr float ct_cosf(long k, long n) { return float(ct_cos2pi(k, n, false)); }
constexpr float ct_sinf(long k, long n) { return float(ct_cos2pi(k, n, true)); }

constexpr int ct_modinv(int a, int m)
{
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}

constexpr int ct_gcd(int a, int b) { return b == 0 ? a : ct_gcd(b, a % b); }

// compile-time loop: f(std::integral_constant<int, i>) for i in [B, E)
template <int B, int E, class F>
BT_HD void static_for(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// a * exp(+j 2 pi K / N) for compile-time K, N
template <long K_, long N_>
BT_HD c32 rot(c32 a)
{
    constexpr long k = ((K_ % N_) + N_) % N_;
    constexpr float h = 0.707106781186547524400844362104849039f;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (2 * k == N_) {
        return -a;
    } else if constexpr (4 * k == N_) {
        return mul_j(a);
    } else if constexpr (4 * k == 3 * N_) {
        return -mul_j(a);
    } else if constexpr (8 * k == N_) {
        return c32{(a.x - a.y) * h, (a.x + a.y) * h};
    } else if constexpr (8 * k == 3 * N_) {
        return c32{(-a.x - a.y) * h, (a.x - a.y) * h};
    } else if constexpr (8 * k == 5 * N_) {
        return c32{(a.y - a.x) * h, (-a.x - a.y) * h};
    } else if constexpr (8 * k == 7 * N_) {
        return c32{(a.x + a.y) * h, (a.y - a.x) * h};
    } else {
        constexpr float c = ct_cosf(k, N_), s = ct_sinf(k, N_);
        return c32{a.x * c - a.y * s, a.x * s + a.y * c};
    }
}

template <int R>
BT_HD void dft(c32 (&v)[R]);

// ------------------------------------------------------------------ radix 2 and 4
BT_HD void dft2(c32 (&v)[2])
{
    c32 a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

BT_HD void dft4(c32 (&v)[4])
{
    c32 s02 = v[0] + v[2], d02 = v[0] - v[2];
    c32 s13 = v[1] + v[3], d13 = mul_j(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
}

// ------------------------------------------------------------------ odd R, symmetric pairs
// X_m = v0 + sum_r (v_r + v_{R-r}) cos(2 pi r m/R) + j sum_r (v_r - v_{R-r}) sin(2 pi r m/R)
template <int R>
BT_HD void dft_odd(c32 (&v)[R])
{
    constexpr int H = (R - 1) / 2;
    c32 a[H], b[H];
    static_for<1, H + 1>([&](auto rI) {
        constexpr int r = decltype(rI)::value;
        a[r - 1] = v[r] + v[R - r];
        b[r - 1] = v[r] - v[R - r];
    });
    const c32 x0 = v[0];
    c32 sum = x0;
    static_for<0, H>([&](auto rI) { sum = sum + a[decltype(rI)::value]; });
    static_for<1, H + 1>([&](auto mI) {
        constexpr int m = decltype(mI)::value;
        c32 re = x0, im = c32{0.f, 0.f};
        static_for<1, H + 1>([&](auto rI) {
            constexpr int r = decltype(rI)::value;
            constexpr float c = ct_cosf((long)r * m, R), s = ct_sinf((long)r * m, R);
            re.x += a[r - 1].x * c;
            re.y += a[r - 1].y * c;
            if constexpr (r == 1) {
                im.x = b[0].x * s;
                im.y = b[0].y * s;
            } else {
                im.x += b[r - 1].x * s;
                im.y += b[r - 1].y * s;
            }
        });
        const c32 jim = mul_j(im);
        v[m] = re + jim;
        v[R - m] = re - jim;
    });
    v[0] = sum;
}

// ------------------------------------------------------------------ Cooley-Tukey R = A B
// n = n1 + A n2, k = B k1 + k2: B-point DFTs over n2, twiddle w_R^{n1 k2}, A-point DFTs over n1
template <int A, int B>
BT_HD void dft_ct(c32 (&v)[A * B])
{
    constexpr int R = A * B;
    c32 y[A][B];
    static_for<0, A>([&](auto n1I) {
        constexpr int n1 = decltype(n1I)::value;
        c32 t[B];
        static_for<0, B>([&](auto n2I) { t[decltype(n2I)::value] = v[n1 + A * decltype(n2I)::value]; });
        dft<B>(t);
        static_for<0, B>([&](auto k2I) {
            constexpr int k2 = decltype(k2I)::value;
            y[n1][k2] = rot<(long)n1 * k2, R>(t[k2]);
        });
    });
    static_for<0, B>([&](auto k2I) {
        constexpr int k2 = decltype(k2I)::value;
        c32 t[A];
        static_for<0, A>([&](auto n1I) { t[decltype(n1I)::value] = y[decltype(n1I)::value][k2]; });
        dft<A>(t);
        static_for<0, A>([&](auto k1I) { v[B * decltype(k1I)::value + k2] = t[decltype(k1I)::value]; });
    });
}

// ------------------------------------------------------------------ Good-Thomas R = A B, gcd 1
// input n = (B n1 + A n2) mod R, output k = (B tB k1 + A tA k2) mod R with
// tB = B^{-1} mod A, tA = A^{-1} mod B; then w_R^{nk} = w_A^{n1 k1} w_B^{n2 k2}
template <int A, int B>
BT_HD void dft_pfa(c32 (&v)[A * B])
{
    constexpr int R = A * B;
    static_assert(ct_gcd(A, B) == 1, "prime-factor map needs coprime factors");
    constexpr int tB = ct_modinv(B % A, A);
    constexpr int tA = ct_modinv(A % B, B);
    c32 y[A][B];
    static_for<0, A>([&](auto n1I) {
        constexpr int n1 = decltype(n1I)::value;
        c32 t[B];
        static_for<0, B>([&](auto n2I) {
            constexpr int n2 = decltype(n2I)::value;
            t[n2] = v[(B * n1 + A * n2) % R];
        });
        dft<B>(t);
        static_for<0, B>([&](auto k2I) { y[n1][decltype(k2I)::value] = t[decltype(k2I)::value]; });
    });
    static_for<0, B>([&](auto k2I) {
        constexpr int k2 = decltype(k2I)::value;
        c32 t[A];
        static_for<0, A>([&](auto n1I) { t[decltype(n1I)::value] = y[decltype(n1I)::value][k2]; });
        dft<A>(t);
        static_for<0, A>([&](auto k1I) {
            constexpr int k1 = decltype(k1I)::value;
            v[(B * tB * k1 + A * tA * k2) % R] = t[k1];
        });
    });
}

template <int R>
BT_HD void dft(c32 (&v)[R])
{
    if constexpr (R == 1) {
        (void)v;
    } else if constexpr (R == 2) {
        dft2(v);
    } else if constexpr (R == 4) {
        dft4(v);
    } else if constexpr (R == 8) {
        dft_ct<2, 4>(v);
    } else if constexpr (R == 16) {
        dft_ct<4, 4>(v);
    } else if constexpr (R == 32) {
        dft_ct<4, 8>(v);
    } else if constexpr (R == 64) {
        dft_ct<8, 8>(v);
    } else if constexpr (R == 6) {
        dft_pfa<2, 3>(v);
    } else if constexpr (R == 10) {
        dft_pfa<2, 5>(v);
    } else if constexpr (R == 12) {
        dft_pfa<4, 3>(v);
    } else if constexpr (R == 14) {
        dft_pfa<2, 7>(v);
    } else if constexpr (R == 15) {
        dft_pfa<3, 5>(v);
    } else if constexpr (R % 2 == 1) {
        dft_odd<R>(v);
    } else {
        static_assert(R % 2 == 1, "unsupported radix");
    }
}

} // namespace bt
