// pow_fp64.h -- x^y for FP32 operands with C99 pow semantics (Annex F),
// computed in FP64 and rounded to FP32 once.
//
// On gfx950 an FP64 add, multiply or FMA issues at the rate of a
// non-packed FP32 one, so carrying the computation in FP64 with short
// textbook series is both cheaper than an FP32 pow built from double-float
// pieces and more accurate (the FP64 result is within about 1e-12 relative
// of x^y, so the FP32 result is the correctly rounded one except when x^y
// lies within that distance of a rounding boundary, where it can be 1 ulp
// off):
//   log2|x| = e + 2 atanh(s) / ln 2 with |x| = m 2^e, m in [sqrt(1/2),
//     sqrt(2)), s = (m - 1) / (m + 1), |s| <= 0.1716, and 2 atanh(s) =
//     2 s (1 + s^2/3 + s^4/5 + ... + s^14/15) (truncation below 4e-14);
//   2^t = 2^n e^g with n = rint(t), g = (t - n) ln 2, |g| <= 0.347, and e^g
//     by its Taylor polynomial to degree 10 (truncation below 3e-13);
//   t is clamped to [-200, 200], beyond which the FP32 result is 0 or inf.
// The function is plain C++ on doubles so that it can also be compiled for
// the host and checked against the C library there.
#pragma once

#include <math.h>
#include <stdint.h>

#ifndef TGP_HD
#ifdef __HIPCC__
#define TGP_HD __host__ __device__
#else
#define TGP_HD
#endif
#endif

namespace tgp {

// fma(a, b, c) for a constant c.  On the device the addend is kept in scalar
// registers and the three-operand FP64 FMA is used directly: the compiler's
// own choice, the two-operand form that accumulates into its destination,
// first copies the constant into vector registers (two extra VALU moves per
// polynomial term and case).  The result is the same correctly rounded FMA.
TGP_HD inline double fma_k(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
#else
    return fma(a, b, c);
#endif
}

TGP_HD inline double log2_fp64(double ax) {  // ax > 0, finite
    int e;
    double m = frexp(ax, &e);  // m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double p = 1.0 / 15.0;
    p = fma_k(p, z, 1.0 / 13.0);
    p = fma_k(p, z, 1.0 / 11.0);
    p = fma_k(p, z, 1.0 / 9.0);
    p = fma_k(p, z, 1.0 / 7.0);
    p = fma_k(p, z, 1.0 / 5.0);
    p = fma_k(p, z, 1.0 / 3.0);
    const double s2 = 2.0 * s;  // exact
    const double ln_m = fma(s2, z * p, s2);
    return fma(ln_m, 1.44269504088896340736, (double)e);  // 1 / ln 2
}

TGP_HD inline double exp2_fp64(double t) {
    t = t > 200.0 ? 200.0 : (t < -200.0 ? -200.0 : t);
    const double n = rint(t);
    const double g = (t - n) * 0.69314718055994530942;  // ln 2
    double p = 1.0 / 3628800.0;  // 1/10!
    p = fma_k(p, g, 1.0 / 362880.0);
    p = fma_k(p, g, 1.0 / 40320.0);
    p = fma_k(p, g, 1.0 / 5040.0);
    p = fma_k(p, g, 1.0 / 720.0);
    p = fma_k(p, g, 1.0 / 120.0);
    p = fma_k(p, g, 1.0 / 24.0);
    p = fma_k(p, g, 1.0 / 6.0);
    p = fma_k(p, g, 0.5);
    p = fma(p, g, 1.0);
    p = fma(p, g, 1.0);
    return ldexp(p, (int)n);
}

// C99 pow on FP32 operands.
TGP_HD inline float pow_fp64(float x, float y) {
    const float ax = fabsf(x), ay = fabsf(y);
    const bool y_int = ay < INFINITY && y == rintf(y);
    // every FP32 value of magnitude >= 2^24 is even
    const bool y_odd = y_int && ay < 16777216.0f && ((int32_t)y & 1) != 0;
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
    if (x < 0.0f && !y_int) return __builtin_nanf("");
    const float r = (float)exp2_fp64((double)y * log2_fp64((double)ax));
    return x < 0.0f && y_odd ? -r : r;
}

}  // namespace tgp
