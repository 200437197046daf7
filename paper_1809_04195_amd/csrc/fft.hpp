// fft.hpp -- mixed-radix complex FFT building blocks for gfx950 (also compilable
// as plain C++ so the codelets and the two-step plans can be checked on a CPU).
//
// Transforms are unnormalised: forward X[k] = sum_n x[n] W_L^{nk}, W_L = exp(-2 pi i / L);
// inverse uses W_L^{-nk}.  Small DFTs run in registers: radix 2/3/4/5 codelets, odd
// prime radices (13) by the symmetric direct sum, composites by Cooley-Tukey, all with
// compile-time twiddles; a length-L transform is a two-step plan L = R1 R2 across the
// threads of one transform with one LDS exchange (RegPlan / RowPlan below), with the
// inter-step twiddles W_L^m from a table (LDS on the GPU).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define T2S_HD __host__ __device__
#define T2S_INL __forceinline__
#else
#include <cstdint>
#define T2S_HD
#define T2S_INL inline
struct float2 {
    float x, y;
};
static inline float2 make_float2(float a, float b) { return float2{a, b}; }
#endif

namespace t2s {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
T2S_HD T2S_INL float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
T2S_HD T2S_INL float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
T2S_HD T2S_INL float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
T2S_HD T2S_INL float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
T2S_HD T2S_INL float2 conjc(float2 a) { return make_float2(a.x, -a.y); }
T2S_HD T2S_INL float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
T2S_HD T2S_INL float2 mul_minus_i(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)
T2S_HD T2S_INL float2 mul_plus_i(float2 a) { return make_float2(-a.y, a.x); }    // a * (+i)

// ---------------------------------------------------------------------------
// compile-time roots of unity (double precision Taylor series after reduction
// of the angle into [-pi/2, pi/2])
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int i = 1; i < 18; ++i) {
        t *= -x * x / double((2 * i) * (2 * i + 1));
        s += t;
    }
    return s;
}
constexpr double taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int i = 1; i < 18; ++i) {
        t *= -x * x / double((2 * i - 1) * (2 * i));
        s += t;
    }
    return s;
}

struct cplxd {
    double re, im;
};

// exp(-2 pi i m / n)
constexpr cplxd root_of_unity(long m, long n) {
    m %= n;
    if (m < 0) m += n;
    if ((4 * m) % n == 0) {
        const long q = (4 * m) / n;  // quarter turns
        if (q == 0) return cplxd{1.0, 0.0};
        if (q == 1) return cplxd{0.0, -1.0};
        if (q == 2) return cplxd{-1.0, 0.0};
        return cplxd{0.0, 1.0};
    }
    double th = (2 * m > n) ? -2.0 * kPi * double(n - m) / double(n) : 2.0 * kPi * double(m) / double(n);
    double s = 0.0, c = 0.0;
    if (th > kPi / 2) {
        const double p = kPi - th;
        s = taylor_sin(p);
        c = -taylor_cos(p);
    } else if (th < -kPi / 2) {
        const double p = -kPi - th;
        s = taylor_sin(p);
        c = -taylor_cos(p);
    } else {
        s = taylor_sin(th);
        c = taylor_cos(th);
    }
    return cplxd{c, -s};
}

template <int R>
struct RootTable {
    float re[R];
    float im[R];
    constexpr RootTable() : re(), im() {
        for (int m = 0; m < R; ++m) {
            const cplxd w = root_of_unity(m, R);
            re[m] = float(w.re);
            im[m] = float(w.im);
        }
    }
};

// x * W_R^e for a compile-time-constant (after unrolling) exponent e
template <int R>
T2S_HD T2S_INL float2 tw_const(float2 x, int e) {
    e %= R;
    if (e == 0) return x;
    if (4 * e == R) return mul_minus_i(x);
    if (2 * e == R) return make_float2(-x.x, -x.y);
    if (4 * e == 3 * R) return mul_plus_i(x);
    constexpr RootTable<R> T{};
    return cmul(x, make_float2(T.re[e], T.im[e]));
}

constexpr int first_factor(int R) {
    return (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3 : (R % 5 == 0 && R != 5) ? 5 : R;
}

// ---------------------------------------------------------------------------
// forward DFT codelets, in registers
// ---------------------------------------------------------------------------
template <int R>
T2S_HD T2S_INL void dft(float2 (&v)[R]);

template <int R>
T2S_HD T2S_INL void dft_base(float2 (&v)[R]) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        constexpr float s3 = 0.866025403784438646763723170752936183f;  // sin(2 pi / 3)
        const float2 t = cadd(v[1], v[2]);
        const float2 d = csub(v[1], v[2]);
        const float2 m = make_float2(v[0].x - 0.5f * t.x, v[0].y - 0.5f * t.y);
        const float2 q = make_float2(s3 * d.y, -s3 * d.x);  // -i s3 d
        v[0] = cadd(v[0], t);
        v[1] = cadd(m, q);
        v[2] = csub(m, q);
    } else if constexpr (R == 4) {
        const float2 t0 = cadd(v[0], v[2]);
        const float2 t1 = csub(v[0], v[2]);
        const float2 t2 = cadd(v[1], v[3]);
        const float2 t3 = mul_minus_i(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    } else if constexpr (R == 5) {
        constexpr float c1 = 0.309016994374947424102293417182819059f;   // cos(2 pi / 5)
        constexpr float c2 = -0.809016994374947424102293417182819059f;  // cos(4 pi / 5)
        constexpr float s1 = 0.951056516295153572116439333379382143f;   // sin(2 pi / 5)
        constexpr float s2 = 0.587785252292473129168705954639072769f;   // sin(4 pi / 5)
        const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
        const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
        const float2 x0 = v[0];
        const float2 m1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        const float2 m2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        const float2 n1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
        const float2 n2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
        v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
        v[1] = cadd(m1, mul_minus_i(n1));
        v[4] = cadd(m1, mul_plus_i(n1));
        v[2] = cadd(m2, mul_minus_i(n2));
        v[3] = cadd(m2, mul_plus_i(n2));
    } else {
        // odd prime R >= 7: with a_n = x_n + x_(R-n), b_n = x_n - x_(R-n) (n = 1..(R-1)/2),
        // X_k = x_0 + sum_n a_n cos(2 pi n k / R) - i sum_n b_n sin(2 pi n k / R) and
        // X_(R-k) the same with +i
        static_assert(R % 2 == 1, "direct codelet for odd radices only");
        constexpr int H = (R - 1) / 2;
        constexpr RootTable<R> T{};   // T.re = cos, T.im = -sin of 2 pi m / R
        float2 a[H + 1], b[H + 1];
#pragma unroll
        for (int n = 1; n <= H; ++n) {
            a[n] = cadd(v[n], v[R - n]);
            b[n] = csub(v[n], v[R - n]);
        }
        float2 X[R];
        float2 s0 = v[0];
#pragma unroll
        for (int n = 1; n <= H; ++n) s0 = cadd(s0, a[n]);
        X[0] = s0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            float2 A = v[0], Bs = make_float2(0.f, 0.f);
#pragma unroll
            for (int n = 1; n <= H; ++n) {
                const int e = (n * k) % R;
                const float c = T.re[e], sn = -T.im[e];
                A = make_float2(A.x + c * a[n].x, A.y + c * a[n].y);
                Bs = make_float2(Bs.x + sn * b[n].x, Bs.y + sn * b[n].y);
            }
            X[k] = cadd(A, mul_minus_i(Bs));
            X[R - k] = cadd(A, mul_plus_i(Bs));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = X[r];
    }
}

// R = A * B: n = B n1 + n2, k = k1 + A k2
template <int R>
T2S_HD T2S_INL void dft(float2 (&v)[R]) {
    constexpr int A = first_factor(R);
    if constexpr (A == R) {
        dft_base<R>(v);
    } else {
        constexpr int B = R / A;
        float2 Y[R];
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) {
            float2 a[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) a[n1] = v[B * n1 + n2];
            dft<A>(a);
#pragma unroll
            for (int k1 = 0; k1 < A; ++k1) Y[n2 * A + k1] = tw_const<R>(a[k1], n2 * k1);
        }
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
            float2 b[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) b[n2] = Y[n2 * A + k1];
            dft<B>(b);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = b[k2];
        }
    }
}

template <int R, bool INV>
T2S_HD T2S_INL void dft_dir(float2 (&v)[R]) {
    if constexpr (INV) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r].y = -v[r].y;
        dft<R>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) v[r].y = -v[r].y;
    } else {
        dft<R>(v);
    }
}

// ---------------------------------------------------------------------------
// supported lengths: a column length (passes B and the readout transform, whose
// thread layout needs R2 | 16 and ny a multiple of 16) or a row length (passes A and C)
// ---------------------------------------------------------------------------
constexpr bool fft_col_length_supported(int L) {
    return L == 16 || L == 32 || L == 48 || L == 64 || L == 96 || L == 128 || L == 160 || L == 192 ||
           L == 240 || L == 256 || L == 320 || L == 384 || L == 512;
}
constexpr bool fft_row_length_supported(int L) { return fft_col_length_supported(L) || L == 260; }

// ---------------------------------------------------------------------------
// Two-step ("four-step") register plans: L = R1 * R2.
//   forward step 1: thread n2 < R2 holds x[R2 n1 + n2] (n1 < R1), DFT_R1, then
//                   multiplies output k1 by W_L^(n2 k1) and writes it to an LDS
//                   exchange slot (k1, n2);
//   forward step 3: thread k1 < R1 reads slots (k1, n2 < R2), DFT_R2, and holds
//                   X[k1 + R1 k2] (k2 < R2).
//   inverse step 1: thread k1 < R1 holds X[k1 + R1 k2], inverse DFT_R2, multiplies
//                   output m1 by W_L^-(k1 m1), writes slot (m1, k1);
//   inverse step 3: thread m1 < R2 reads slots (m1, k1 < R1), inverse DFT_R1, and
//                   holds x[m1 + R2 m2] (m2 < R1).
// So each transform crosses LDS once, and a forward transform followed by an
// inverse one needs no exchange in between (the frequency-side layouts match).
// ---------------------------------------------------------------------------
template <int L>
struct RegPlan;
template <> struct RegPlan<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct RegPlan<32> { static constexpr int R1 = 4, R2 = 8; };
template <> struct RegPlan<48> { static constexpr int R1 = 6, R2 = 8; };
template <> struct RegPlan<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct RegPlan<96> { static constexpr int R1 = 12, R2 = 8; };
template <> struct RegPlan<128> { static constexpr int R1 = 8, R2 = 16; };
template <> struct RegPlan<160> { static constexpr int R1 = 10, R2 = 16; };
template <> struct RegPlan<192> { static constexpr int R1 = 12, R2 = 16; };
template <> struct RegPlan<240> { static constexpr int R1 = 15, R2 = 16; };
template <> struct RegPlan<256> { static constexpr int R1 = 16, R2 = 16; };
template <> struct RegPlan<320> { static constexpr int R1 = 20, R2 = 16; };
template <> struct RegPlan<384> { static constexpr int R1 = 24, R2 = 16; };
template <> struct RegPlan<512> { static constexpr int R1 = 32, R2 = 16; };

// Plan of the row passes (A and C), which transform rows of length nz: the same as
// RegPlan except at 384, where 16 x 24 puts all 24 threads of a row to work in the
// row-major phase (coil-map loads, accumulation) and holds 16 values per thread
// there instead of 24.
template <int L>
struct RowPlan : RegPlan<L> {};
template <> struct RowPlan<384> { static constexpr int R1 = 16, R2 = 24; };
// 260 = 13 x 20 (radix-13 codelet), a row length only (260 is not a multiple of 16)
template <> struct RowPlan<260> { static constexpr int R1 = 13, R2 = 20; };

template <int L, class Plan = RegPlan<L>>
struct RegGeom {
    static constexpr int R1 = Plan::R1;
    static constexpr int R2 = Plan::R2;
    static_assert(R1 * R2 == L, "plan does not factor L");
    static constexpr int P = R1 > R2 ? R1 : R2;              // threads per transform
    static constexpr int S1 = R2 + 1;                         // forward slot stride (k1 rows)
    static constexpr int S2 = R1 + 1;                         // inverse slot stride (m1 rows)
    static constexpr int TB0 = R1 * R2 + P;                   // >= R1 * S1 and >= R2 * S2
    static constexpr int TB = TB0 + ((17 - TB0 % 16) % 16);   // per-transform LDS words, == 1 mod 16
};


}  // namespace t2s
