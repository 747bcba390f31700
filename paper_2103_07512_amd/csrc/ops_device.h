// ops_device.h -- FP32 device implementations of the primitive set (Table 1).
//
// Every operator maps FP32 operands to one FP32 result.  Protected forms
// follow Table 1 of the paper; the readings where the table is silent are
// the ones documented in include/tgp.h.  The same functions serve the fused
// interpreter, the cache fill and the evaluate path, and the library is
// compiled with -ffp-contract=off, so a subtree gives bit-identical values
// whichever path computes it.
#pragma once

#include <hip/hip_runtime.h>

#include "fp32_math.h"

namespace tgp {

__device__ __forceinline__ float f_add(float a, float b) { return a + b; }
__device__ __forceinline__ float f_sub(float a, float b) { return a - b; }
__device__ __forceinline__ float f_mult(float a, float b) { return a * b; }
// Operators with a fast path and a general one: *_fast computes the common
// case without branches and says whether its value stands (ok); f_op takes
// the general form only for the cases left, so a wave branches once per case
// and skips the general code when no lane needs it.

// Correctly rounded IEEE division; 0 for a zero denominator of either sign.
__device__ __forceinline__ float f_div(float a, float b) { return b == 0.0f ? 0.0f : a / b; }
// sin(pi x), cos(pi x), tan(pi x) in FP32 (fp32_math.h): exact quarter-
// period reduction, minimax polynomials; exact at every multiple of 1/2,
// zeros returned as +0.
__device__ __forceinline__ float f_sin(float a) { return sinpi_f32(a); }
__device__ __forceinline__ float f_cos(float a) { return cospi_f32(a); }
__device__ __forceinline__ float f_tan(float a) { return tanpi_f32(a); }
// e^x: for |x| < 87 (a normal result) 2^t with t = x log2(e) carried as a
// double-FP32 sum (the product split exactly by fma, plus x times the low
// part of log2(e)), 2^t = 2^t_hi (1 + t_lo ln 2) from the hardware exp2
// (within 0.77 ulp): within 1.3 ulp.  Other arguments take the library's
// expf (overflow, subnormal results, NaN).
__device__ __forceinline__ float exp_fast(float a, bool &ok) {
    const float th = a * 0x1.715476p+0f;
    const float tl = fmaf(a, 0x1.715476p+0f, -th) + a * 0x1.4ae0c0p-26f;
    const float r = __builtin_amdgcn_exp2f(th);
    ok = fabsf(a) < 87.0f;
    return fmaf(r, tl * 0x1.62e430p-1f, r);
}
__device__ __forceinline__ float f_exp(float a) {
    bool ok;
    const float r = exp_fast(a, ok);
    return ok ? r : expf(a);
}
// Protected log: -1 for a negative argument.  A positive normal argument
// takes the hardware log2 (within one ulp) times ln 2 split in two FP32
// parts: within 1.5 ulp of the result's relative error bound 2^-21.  Zero,
// subnormals, infinity and NaN take the library's logf.
__device__ __forceinline__ float log_fast(float a, bool &ok) {
    const float l2 = __builtin_amdgcn_logf(a);
    ok = (a < 0.0f) | ((a >= 0x1p-126f) & (a < __builtin_inff()));
    return a < 0.0f ? -1.0f : fmaf(l2, 0x1.62e430p-1f, l2 * -0x1.05c610p-29f);
}
__device__ __forceinline__ float f_log(float a) {
    bool ok;
    const float r = log_fast(a, ok);
    return ok ? r : logf(a);
}
// x^y with 0^0 = 0, otherwise C99 pow.  The common case -- a finite
// nonzero base (positive, or negative with an integer exponent), |y| <= 2,
// and a result in the normal range -- goes through the hardware base-2
// logarithm and exponential (v_log_f32, v_exp_f32; both within one ulp,
// v_log_f32 measured exhaustively over [0.70, 1.42]): x = 2^e m with m in
// [sqrt(1/2), sqrt(2)), t = y e + y log2(m) is carried as a double-FP32 sum
// (the products split exactly by fma, the sum by TwoSum), and
// 2^t = 2^t_hi (1 + t_lo ln 2).  The error of log2(m) (at most 2^-24.37)
// times |y| <= 2, the exponential's ulp and the last rounding keep the
// result within 2.4 ulp.  A finite negative base with a finite non-integer
// exponent gives NaN; everything else takes pow_f32 (fp32_math.h).
__device__ __forceinline__ float pow_fast(float a, float b, bool &ok) {
    const float ax = fabsf(a), ab = fabsf(b);
    const bool yint = rintf(b) == b;
    const bool nan_case = (a < 0.0f) & (ax < __builtin_inff()) & !yint & (ab < __builtin_inff());
    float m = __builtin_amdgcn_frexp_mantf(ax);
    int e = __builtin_amdgcn_frexp_expf(ax);
    const bool lo = m < 0.70710678f;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const float fe = (float)e;
    const float lm = __builtin_amdgcn_logf(m);
    const float p = b * fe, pe = fmaf(b, fe, -p);
    const float q = b * lm, qe = fmaf(b, lm, -q);
    const float th = p + q;
    const float bb = th - p;
    const float tl = ((p - (th - bb)) + (q - bb)) + (pe + qe);
    float r = __builtin_amdgcn_exp2f(th);
    r = fmaf(r, tl * 0x1.62e430p-1f, r);
    r = ((a < 0.0f) & (ab == 1.0f)) ? -r : r;
    ok = nan_case | ((ab <= 2.0f) & (ax > 0.0f) & (ax < __builtin_inff()) & (th >= -125.0f) & (th <= 127.0f));
    return nan_case ? __builtin_nanf("") : r;
}
__device__ __forceinline__ float f_pow(float a, float b) {
    bool ok;
    const float r = pow_fast(a, b, ok);
    return ok ? r : ((a == 0.0f && b == 0.0f) ? 0.0f : pow_f32(a, b));
}
// min and max: the hardware's v_min_f32 / v_max_f32, which return the other
// operand when one is a quiet NaN and order -0 below +0 (the reading of
// include/tgp.h).  They differ from fminf / fmaxf only on signalling NaNs,
// and no operand here is one: constants are made quiet where they enter
// (the program emitter, the folding kernel) and every operator returns quiet
// NaNs, so the compiler's quieting of both operands (two more instructions
// per call, as it cannot prove this) is left out.
__device__ __forceinline__ float f_min(float a, float b) {
    float r;
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float f_max(float a, float b) {
    float r;
    asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
// Halving each operand first is exact in the normal range and cannot overflow.
__device__ __forceinline__ float f_mdist(float a, float b) { return a * 0.5f + b * 0.5f; }
__device__ __forceinline__ float f_neg(float a) { return -a; }
// Protected square root (0 below 0): the hardware square root, within 0.93
// ulp and exact on exact squares (measured over every significand of a
// binade); subnormal arguments are scaled by 2^32 first (the result by 2^-16,
// both exact).
__device__ __forceinline__ float f_sqrt(float a) {
    const bool sub = a < 0x1p-126f;
    const float s = __builtin_amdgcn_sqrtf(sub ? a * 0x1p32f : a);
    return a < 0.0f ? 0.0f : (sub ? s * 0x1p-16f : s);
}
__device__ __forceinline__ float f_sign(float a) {
    return a > 0.0f ? 1.0f : (a < 0.0f ? -1.0f : 0.0f);
}
__device__ __forceinline__ float f_abs(float a) { return fabsf(a); }
__device__ __forceinline__ float f_clip(float a, float b, float c) { return f_max(f_min(a, c), b); }
// Floored remainder (the divisor's sign), rounded once from its exact value;
// 0 for a zero divisor of either sign.  The quotient comes from the
// hardware reciprocal (within one ulp) when |a / b| < 2^20 and 2^-125 <= |b|
// <= 2^125: q0 = a rcp(b) is then within 2^-22.5 |a/b| of a/b, raised by
// |q0| 2^-21 it is never below a/b and stays below a/b + 1, so its floor q
// is floor(a/b) or one more.  Either way a - q b lies within |b| of zero and
// the fma gives it exactly, and one more b fixes the sign when q was one
// too many: the same correctly rounded value as floor_mod_f32
// (fp32_math.h), which takes every other operand.
__device__ __forceinline__ float mod_fast(float a, float b, bool &ok) {
    const float ab = fabsf(b);
    const float q0 = a * __builtin_amdgcn_rcpf(b);
    const float q = floorf(fmaf(fabsf(q0), 0x1p-21f, q0));
    float r = fmaf(-q, b, a);
    r = ((r != 0.0f) & ((r < 0.0f) != (b < 0.0f))) ? r + b : r;
    r = r == 0.0f ? copysignf(0.0f, a) : r;
    ok = ((fabsf(q0) < 1048576.0f) & (ab >= 0x1p-125f) & (ab <= 0x1p125f)) | (b == 0.0f);
    return b == 0.0f ? 0.0f : r;
}
__device__ __forceinline__ float f_mod(float a, float b) {
    bool ok;
    const float r = mod_fast(a, b, ok);
    return ok ? r : floor_mod_f32(a, b);
}
__device__ __forceinline__ float f_frac(float a) { return a - floorf(a); }
__device__ __forceinline__ float f_if(float a, float b, float c) { return a != 0.0f ? b : c; }
__device__ __forceinline__ float f_step(float a) { return a < 0.0f ? -1.0f : 1.0f; }
// The image operators in FP32 (fp32_math.h): sstep and sstepp as short
// products, len scaled by a power of two, lerp with exact intermediate parts.
__device__ __forceinline__ float f_sstep(float a) { return sstep_f32(a); }
__device__ __forceinline__ float f_sstepp(float a) { return sstepp_f32(a); }
__device__ __forceinline__ float f_len(float a, float b) { return len_f32(a, b); }
__device__ __forceinline__ float f_lerp(float a, float b, float c) { return lerp_f32(a, b, c); }
// warp: the nearest point of an axis of n points to position (t - lo) *
// scale, halves rounded up, clamped to the axis; NaN gives point 0 (fmaxf
// returns its other operand).
__device__ __forceinline__ int32_t warp_point(float t, float lo, float scale, int32_t n) {
    const float u = (t - lo) * scale + 0.5f;
    return (int32_t)floorf(fminf(fmaxf(u, 0.0f), (float)(n - 1)));
}

// Bitwise operators: each operand becomes a 32-bit integer (NaN -> 0,
// truncation toward zero, saturation to the int32 range), the integer result
// is rounded to FP32; kind 0: or, 1: xor, 2: and.
__device__ __forceinline__ int32_t to_i32(float a) {
    if (!(a == a)) return 0;
    if (a >= 2147483648.0f) return 2147483647;
    if (a <= -2147483648.0f) return -2147483647 - 1;
    return (int32_t)a;
}
__device__ __forceinline__ float f_bitop(float a, float b, uint32_t kind) {
    const int32_t x = to_i32(a), y = to_i32(b);
    const int32_t r = kind == 0 ? (x | y) : (kind == 1 ? (x ^ y) : (x & y));
    return (float)r;
}

}  // namespace tgp
