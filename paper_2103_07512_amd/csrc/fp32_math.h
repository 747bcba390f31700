// fp32_math.h -- FP32 implementations of the operators of Table 1 whose
// value needs more than one correctly rounded FP32 operation: sin(pi x),
// cos(pi x) and tan(pi x) (Sec. 3.2 prescales trigonometric arguments by
// pi), x^y, the floored remainder, and the image operators sstep, sstepp,
// len and lerp.
//
// Everything is FP32 arithmetic: exact range reductions, fused multiply-
// adds, error-free transformations (TwoSum, Fast2Sum, the fma product
// residual) where a result needs more than 24 bits on the way, and minimax
// polynomials whose coefficients come from gen_minimax.py (a Remez exchange
// in FP64, coefficients rounded to FP32).  Each operator is within a few
// half-ulps of the exact value of its FP32 operands; tests/fp32_math_check.cpp
// measures that on the host against the C library in FP64 (the functions are
// plain C++ on floats, so the host runs the same operations as the device).
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#ifndef TGP_HD
#ifdef __HIPCC__
#define TGP_HD __host__ __device__
#else
#define TGP_HD
#endif
#endif

namespace tgp {

TGP_HD inline float bits_to_float(uint32_t u) {
    float f;
    memcpy(&f, &u, sizeof f);
    return f;
}

TGP_HD inline uint32_t float_to_bits(float f) {
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return u;
}

// v with its sign flipped when `flip` is set (bit 31 of the mask).
TGP_HD inline float flip_sign(float v, uint32_t mask) { return bits_to_float(float_to_bits(v) ^ mask); }

// ------------------------------------------------------------- sin / cos
// sin(pi t) = t S(t^2) and cos(pi t) = 1 + t^2 C(t^2) on |t| <= 1/4
// (gen_minimax.py: S of degree 3, C of degree 3, relative error).
constexpr float kS0 = 3.1415927410125732f, kS1 = -5.167707920074463f, kS2 = 2.5497610569000244f,
                kS3 = -0.5890122056007385f;
constexpr float kC0 = -4.934802055358887f, kC1 = 4.0587077140808105f, kC2 = -1.3350505828857422f,
                kC3 = 0.23136423528194427f;

// a = 2k + n/2 + t with integers k, n (n in -2..2) and |t| <= 1/4, all
// exact in FP32: r = a - 2 rint(a/2) is exact (a and 2 rint(a/2) are
// multiples of ulp(a) at most 1 apart; every FP32 value of magnitude
// >= 2^24 is even, so r = 0 there), and t = r - n/2 likewise.  Returns
// sin(pi t) and cos(pi t) and the quadrant q = n mod 4.  A non-finite a
// gives NaN polynomials (and q = 2, unused).
TGP_HD inline void sincospi_core(float a, float &sp, float &cp, uint32_t &q) {
    const float r = fmaf(-2.0f, rintf(0.5f * a), a);
    const float n = rintf(2.0f * r);
    const float t = fmaf(-0.5f, n, r);
    const float z = t * t;
    sp = t * fmaf(fmaf(fmaf(kS3, z, kS2), z, kS1), z, kS0);
    cp = fmaf(z, fmaf(fmaf(fmaf(kC3, z, kC2), z, kC1), z, kC0), 1.0f);
    q = (uint32_t)(int32_t)fmaxf(n, -2.0f) & 3u;  // fmaxf: NaN gives -2, a defined conversion
}

// sin(pi a); zeros are +0 (at a = k exactly; +0 is added last).
TGP_HD inline float sinpi_f32(float a) {
    float sp, cp;
    uint32_t q;
    sincospi_core(a, sp, cp, q);
    const float v = (q & 1u) ? cp : sp;
    return flip_sign(v, (q & 2u) << 30) + 0.0f;
}

// cos(pi a); zeros are +0 (at a = k + 1/2 exactly).
TGP_HD inline float cospi_f32(float a) {
    float sp, cp;
    uint32_t q;
    sincospi_core(a, sp, cp, q);
    const float v = (q & 1u) ? sp : cp;
    return flip_sign(v, ((q + 1u) & 2u) << 30) + 0.0f;
}

// tan(pi a) = sin(pi a) / cos(pi a) with IEEE division (+-inf at the poles).
TGP_HD inline float tanpi_f32(float a) {
    float sp, cp;
    uint32_t q;
    sincospi_core(a, sp, cp, q);
    const float s = flip_sign((q & 1u) ? cp : sp, (q & 2u) << 30) + 0.0f;
    const float c = flip_sign((q & 1u) ? sp : cp, ((q + 1u) & 2u) << 30) + 0.0f;
    return s / c;
}

// ------------------------------------------------------------------- pow
// 2 / ln 2 as a sum of two FP32 values, and 2 / (ln 2 (2k + 1)) for k = 1..5.
constexpr float kK2Hi = 2.885390043258667f, kK2Lo = 3.851926067000022e-08f;
constexpr float kQ3 = 0.9617967009544373f, kQ5 = 0.5770780444145203f, kQ7 = 0.41219857335090637f,
                kQ9 = 0.32059890031814575f, kQ11 = 0.26230818033218384f, kQ13 = 0.22195307910442352f;
// 2^f = 1 + f E(f) on |f| <= 1/2 (gen_minimax.py, E of degree 6).
constexpr float kE0 = 0.6931471824645996f, kE1 = 0.24022650718688965f, kE2 = 0.055504102259874344f,
                kE3 = 0.009618038311600685f, kE4 = 0.0013333935057744384f, kE5 = 0.00015466756303794682f,
                kE6 = 1.5196156709862407e-05f;

// log2(ax) as hi + lo, for finite ax > 0, to about 2^-30 relative.
// ax = m 2^e with m in [sqrt(1/2), sqrt(2)); log2(m) = (2 / ln 2) atanh(s)
// = (2 / ln 2) s (1 + s^2/3 + s^4/5 + ...) with s = (m - 1) / (m + 1),
// |s| <= 0.1716.  s is formed as s0 + s1 from a Newton reciprocal of m + 1
// (itself kept as dh + dl) and the fma residual of the quotient; the leading
// term (2 / ln 2) s is carried as a double-float, the series beyond it (below
// 1% of it) in FP32.
TGP_HD inline void log2_df(float ax, float &hi, float &lo) {
    int e;
    float m = frexpf(ax, &e);  // [1/2, 1), subnormals included
    if (m < 0.7071067690849304f) {
        m += m;
        --e;
    }
    const float u = m - 1.0f;          // exact (Sterbenz)
    const float dh = 2.0f + u;         // m + 1 rounded
    const float dl = (2.0f - dh) + u;  // its rounding error (Fast2Sum, |2| > |u|)
    float r = fmaf(-0.23901599645614624f, dh, 0.985061526298523f);  // 1/dh within 1.5%
    r = fmaf(r, fmaf(-dh, r, 1.0f), r);
    r = fmaf(r, fmaf(-dh, r, 1.0f), r);                              // within 5e-8
    const float s0 = u * r;
    const float s1 = fmaf(-s0, dl, fmaf(-s0, dh, u)) * r;            // s = s0 + s1
    const float z = s0 * s0;
    const float rest = (s0 * z) * fmaf(fmaf(fmaf(fmaf(fmaf(kQ13, z, kQ11), z, kQ9), z, kQ7), z, kQ5), z, kQ3);
    const float p0 = s0 * kK2Hi;
    // s1 (1 + z): the leading term's part of s1 and its first-order share
    // in the series (which was formed from s0 alone)
    const float p1 = fmaf(s0, kK2Hi, -p0) + fmaf(s0, kK2Lo, fmaf(fmaf(s1, z, s1), kK2Hi, rest));
    const float ph = p0 + p1;          // Fast2Sum: |p0| > |p1| (the rest is below 1%)
    const float pl = p1 - (ph - p0);
    const float fe = (float)e;
    hi = fe + ph;                      // Fast2Sum: |e| >= 1 > |ph|, or e = 0
    lo = (ph - (hi - fe)) + pl;
}

// |x|^y for finite x != 0, 1 and finite y != 0: 2^t with t = y log2|x|
// carried as hi + lo; 2^t = 2^n 2^f with n = rint(t) and |f| <= 1/2 + tiny.
TGP_HD inline float pow_core(float ax, float y) {
    float th, tl;
    log2_df(ax, th, tl);
    const float h0 = y * th;
    const float l0 = fmaf(y, th, -h0) + y * tl;  // t = h0 + l0
    // beyond +-200, 2^t is 0 or inf in FP32: clamp, and drop the low part
    // (it is meaningless there, or NaN when y th overflowed)
    const float h = fminf(fmaxf(h0, -200.0f), 200.0f);
    const float l = h == h0 ? l0 : 0.0f;
    const float n = rintf(h);
    const float f = (h - n) + l;              // h - n exact
    const float p = fmaf(f, fmaf(fmaf(fmaf(fmaf(fmaf(fmaf(kE6, f, kE5), f, kE4), f, kE3), f, kE2), f, kE1), f, kE0),
                         1.0f);
    // 2^n p in two steps, so that n's full range stays within the exponent
    const int ni = (int)n;
    const int n1 = ni / 2;
    return ldexpf(ldexpf(p, n1), ni - n1);
}

// C99 pow on FP32 operands (Annex F special cases), computed in FP32.
// The common case (x finite, nonzero, not 1; y finite, nonzero; an
// integral y when x < 0) takes one path; results within about 4 half-ulps.
TGP_HD inline float pow_f32(float x, float y) {
    const float ax = fabsf(x), ay = fabsf(y);
    const bool y_int = y == rintf(y);         // false for NaN; true for +-inf
    // every FP32 value of magnitude >= 2^24 is even
    const bool y_odd = y_int && ay < 16777216.0f && ((int32_t)y & 1) != 0;
    if (ax > 0.0f && ax < INFINITY && ay < INFINITY && y != 0.0f && x != 1.0f && (x > 0.0f || y_int)) {
        const float r = pow_core(ax, y);
        return x < 0.0f && y_odd ? -r : r;
    }
    if (y == 0.0f || x == 1.0f) return 1.0f;  // even when the other operand is NaN
    if (x != x || y != y) return x + y;       // NaN
    if (ay == INFINITY) {
        if (ax == 1.0f) return 1.0f;          // (-1)^(+-inf)
        return (ax < 1.0f) == (y < 0.0f) ? INFINITY : 0.0f;
    }
    if (x == 0.0f) {
        if (y < 0.0f) return y_odd ? copysignf(INFINITY, x) : INFINITY;
        return y_odd ? x : 0.0f;
    }
    if (ax == INFINITY) {
        if (x > 0.0f) return y < 0.0f ? 0.0f : INFINITY;
        if (y < 0.0f) return y_odd ? -0.0f : 0.0f;
        return y_odd ? -INFINITY : INFINITY;
    }
    return bits_to_float(0x7fc00000u);        // x < 0 with a non-integral y: NaN
}

// ------------------------------------------------------------------- mod
// The floored remainder of Table 1's mod (the result takes the divisor's
// sign), b != 0: exact.  With q = floor(RN(a / b)) and |a / b| < 2^23, q is
// floor(a / b) or one more (rounding is monotone and the integers there are
// FP32 values), so a - q b has magnitude below |b|, is a multiple of ulp(b)
// or of ulp(a), and the fma gives it exactly; one more b fixes the sign
// when q was one too many.  A zero result takes the sign of a (as fmod's
// does).  Other operands (a quotient of 2^23 or more, a non-finite a or b)
// go through the library's exact fmodf.
TGP_HD inline float floor_mod_f32(float a, float b) {
    const float q = floorf(a / b);
    if (fabsf(q) < 8388608.0f && fabsf(a) < INFINITY && fabsf(b) < INFINITY) {
        float r = fmaf(-q, b, a);
        if (r != 0.0f && ((r < 0.0f) != (b < 0.0f))) r += b;
        return r == 0.0f ? copysignf(0.0f, a) : r;
    }
    float r = fmodf(a, b);
    if (r != 0.0f && ((r < 0.0f) != (b < 0.0f))) r += b;
    return r;
}

// ------------------------------------------------------- image operators
// x^2 (3 - 2x): three roundings of products and one fused difference.
TGP_HD inline float sstep_f32(float x) { return (x * x) * fmaf(-2.0f, x, 3.0f); }

// x^3 (x (6x - 15) + 10) = x^3 (6 (x - 5/4)^2 + 5/8): the second form sums
// two positive terms, so no cancellation magnifies the rounding.
TGP_HD inline float sstepp_f32(float x) {
    const float t = x - 1.25f;
    return ((x * x) * x) * fmaf(t, 6.0f * t, 0.625f);
}

// sqrt(x^2 + y^2): the larger magnitude is scaled into [1/2, 1) by a power
// of two (exact), so neither square overflows or underflows; NaN when an
// operand is NaN, +inf when one is infinite.
TGP_HD inline float len_f32(float x, float y) {
    if (x != x || y != y) return bits_to_float(0x7fc00000u);
    const float a = fabsf(x), b = fabsf(y);
    const float hi = fmaxf(a, b), lo = fminf(a, b);
    if (hi == INFINITY) return INFINITY;
    if (hi == 0.0f) return 0.0f;
    int e;
    (void)frexpf(hi, &e);
    const float hs = ldexpf(hi, -e), ls = ldexpf(lo, -e);
    return ldexpf(sqrtf(fmaf(hs, hs, ls * ls)), e);
}

// s + e = a + b exactly (Knuth's TwoSum).
TGP_HD inline void two_sum_f32(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// x + (y - x) frac(z), the exact value rounded about once: y - x, the
// fraction z - floor(z) and their product are carried exactly (TwoSum and
// the fma product residual) and only the final sum of the parts rounds.
// Operands of magnitude 2^125 and more are scaled by 1/4 (exactly) so that
// nothing overflows on the way; a non-finite operand gives the class of the
// formula's value.
TGP_HD inline float lerp_f32(float x, float y, float z) {
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return fmaf(y - x, z - floorf(z), x);
    const bool big = fmaxf(fabsf(x), fabsf(y)) >= 0x1p125f;
    const float xs = big ? x * 0.25f : x, ys = big ? y * 0.25f : y;
    float fh, fo, dh, dd, sh, so;
    two_sum_f32(z, -floorf(z), fh, fo);  // frac(z) = fh + fo
    two_sum_f32(ys, -xs, dh, dd);        // ys - xs = dh + dd
    const float ph = dh * fh;
    const float pp = fmaf(dh, fh, -ph) + (dh * fo + dd * fh);  // (ys - xs) frac(z) = ph + pp
    two_sum_f32(xs, ph, sh, so);
    const float r = sh + (so + pp);
    return big ? r * 4.0f : r;
}

}  // namespace tgp
