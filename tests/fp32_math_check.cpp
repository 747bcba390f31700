// Host check of the FP32 operator implementations the device uses
// (fp32_math.h, the same source): each against its exact value computed in
// FP64 by the C library, in ulps of the FP32 result, over special values and
// millions of seeded operands; every result must also stay within the
// accuracy the parity classifier assumes of a library operator (2^-21
// relative, with 2^-126 as the floor below the normal range).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <random>

#include "fp32_math.h"

static uint32_t bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

// ulp of the FP32 value nearest x (2^-149 below the normal range)
static double ulp_at(double x) {
    const double a = fabs(x);
    if (a < 0x1p-126) return 0x1p-149;
    int e;
    frexp(a, &e);                    // a = m 2^e, m in [1/2, 1)
    return ldexp(1.0, e - 24);
}

// sin(pi x), cos(pi x) in FP64 with the exact quarter-period reduction
static void sincospi64(double x, double *s, double *c) {
    if (!isfinite(x)) {
        *s = *c = NAN;
        return;
    }
    if (fabs(x) >= 9007199254740992.0) {
        *s = 0.0;
        *c = 1.0;
        return;
    }
    const double n = rint(2.0 * x);
    const double t = x - 0.5 * n;
    const double st = sin(M_PI * t), ct = cos(M_PI * t);
    long q = (long)fmod(n, 4.0);
    if (q < 0) q += 4;
    switch (q) {
    case 0: *s = st;  *c = ct;  break;
    case 1: *s = ct;  *c = -st; break;
    case 2: *s = -st; *c = -ct; break;
    default: *s = -ct; *c = st; break;
    }
}

struct Stat {
    const char *name;
    double max_ulps = 0.0, lib_limit_ratio = 0.0;
    long n = 0, bad = 0;
    double worst_in[3] = {0, 0, 0};

    // got against the exact value want (FP64); limit in ulps
    void add(float got, double want, double limit, float a, float b = 0, float c = 0) {
        ++n;
        if (isnan(want) || isinf(want)) {
            const bool same = isnan(want) ? isnan(got) : (isinf(got) && (got > 0) == (want > 0));
            if (!same && !(isinf(want) && fabs((double)got) >= 3.4028234663852886e38)) {
                if (bad < 8) printf("%s(%a, %a, %a) = %a, want %a\n", name, a, b, c, got, want);
                ++bad;
            }
            return;
        }
        if (isinf(got) || isnan(got)) {
            if (fabs(want) >= 3.4028235677973366e38) return;  // overflows in FP32 too
            if (bad < 8) printf("%s(%a, %a, %a) = %a, want %a\n", name, a, b, c, got, want);
            ++bad;
            return;
        }
        const double err = fabs((double)got - want);
        const double u = err / ulp_at(want);
        // the classifier's library accuracy: 2^-21 max(|want|, 2^-126)
        const double lib = err / (0x1p-21 * fmax(fabs(want), 0x1p-126));
        if (u > max_ulps) {
            max_ulps = u;
            worst_in[0] = a;
            worst_in[1] = b;
            worst_in[2] = c;
        }
        if (lib > lib_limit_ratio) lib_limit_ratio = lib;
        if (u > limit || lib > 1.0) {
            if (bad < 8) printf("%s(%a, %a, %a) = %a, want %.17g (%.3f ulp)\n", name, a, b, c, got, want, u);
            ++bad;
        }
    }
    int report() const {
        printf("%-7s %9ld cases, max %.3f ulp at (%a, %a, %a), max %.3f of the library bound, %ld bad\n", name, n,
               max_ulps, worst_in[0], worst_in[1], worst_in[2], lib_limit_ratio, bad);
        return bad ? 1 : 0;
    }
};

int main() {
    std::mt19937_64 rng(20260);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    int fails = 0;

    // sin(pi x), cos(pi x), tan(pi x)
    Stat ss{"sinpi"}, cs{"cospi"}, ts{"tanpi"};
    auto trig = [&](float a) {
        double s, c;
        sincospi64((double)a, &s, &c);
        ss.add(tgp::sinpi_f32(a), s, 2.0, a);
        cs.add(tgp::cospi_f32(a), c, 2.0, a);
        if (c != 0.0) ts.add(tgp::tanpi_f32(a), s / c, 3.0, a);
    };
    for (int i = 0; i < 6000000; ++i) {
        float a;
        switch (i % 4) {
        case 0: a = (float)(u01(rng) * 8.0 - 4.0); break;                 // a few periods
        case 1: a = (float)((u01(rng) - 0.5) * 1e-3); break;              // near 0: relative accuracy
        case 2: a = (float)((u01(rng) - 0.5) * 2e7); break;               // large arguments
        default: a = (float)(rint(u01(rng) * 64 - 32) * 0.5 + (u01(rng) - 0.5) * 1e-4); break;  // near zeros
        }
        trig(a);
    }
    // exact values at every half-integer, zeros as +0
    for (int k = -64; k <= 64; ++k) {
        const float a = 0.5f * (float)k;
        const float s = tgp::sinpi_f32(a), c = tgp::cospi_f32(a);
        double s64, c64;
        sincospi64(a, &s64, &c64);
        if ((double)s != s64 || (double)c != c64 || (s == 0.0f && bits(s) != 0) || (c == 0.0f && bits(c) != 0)) {
            printf("half-integer %g: sin %a cos %a\n", a, s, c);
            ++fails;
        }
    }
    for (float a : {INFINITY, -INFINITY, NAN})
        if (!isnan(tgp::sinpi_f32(a)) || !isnan(tgp::cospi_f32(a))) {
            printf("non-finite argument %a\n", a);
            ++fails;
        }
    for (float a : {16777216.0f, 16777218.0f, 3.0e38f, -3.0e38f, 8388609.0f})
        trig(a);

    // pow: C99 special cases against the C library's powf, bit for bit
    Stat ps{"pow"};
    const float sv[] = {0.0f, -0.0f, 1.0f, -1.0f, 0.5f, -0.5f, 2.0f, -2.0f, 3.0f, -3.0f, 2.5f, -2.5f,
                        INFINITY, -INFINITY, NAN, 16777216.0f, -16777216.0f, 1e-45f, -1e-45f,
                        3.4e38f, -3.4e38f, 1.0000001f, 0.99999994f, 127.0f, -149.0f, 150.0f, -150.5f};
    for (float x : sv)
        for (float y : sv) {
            const float got = tgp::pow_f32(x, y), want = powf(x, y);
            const bool special = x == 0.0f || y == 0.0f || !isfinite(x) || !isfinite(y) || x == 1.0f ||
                                 (x < 0.0f && y != rintf(y));
            if (special) {
                const bool ok = (got != got && want != want) || bits(got) == bits(want);
                if (!ok) {
                    printf("special pow(%a, %a) = %a, libm %a\n", x, y, got, want);
                    ++fails;
                }
            } else {
                ps.add(got, pow((double)x, (double)y), 3.0, x, y);
            }
        }
    for (int i = 0; i < 8000000; ++i) {
        float x, y;
        switch (i % 5) {
        case 0: x = (float)(u01(rng) * 4.0 - 2.0); y = (float)(u01(rng) * 8.0 - 4.0); break;
        case 1: x = (float)exp(u01(rng) * 60.0 - 30.0); y = (float)(u01(rng) * 20.0 - 10.0); break;
        case 2: x = (float)(1.0 + (u01(rng) - 0.5) * 1e-3); y = (float)((u01(rng) - 0.5) * 2e5); break;
        case 3: x = (float)(-(u01(rng) * 10.0)); y = (float)(int)(u01(rng) * 40.0 - 20.0); break;
        default:  // results near overflow and deep in the subnormal range
            x = (float)exp(u01(rng) * 4.0 - 2.0);
            y = (float)((u01(rng) < 0.5 ? 1.0 : -1.0) * (90.0 + u01(rng) * 60.0) / log(fmax(fabs(log((double)x)), 1e-3)));
            break;
        }
        ps.add(tgp::pow_f32(x, y), pow((double)x, (double)y), 3.0, x, y);
    }

    // floored mod: bit for bit the exact floored remainder rounded once
    // (fmod in FP64 of FP32 operands is exact; moving it into the divisor's
    // sign is one FP64 addition, exact too, then one rounding to FP32)
    long mod_n = 0, mod_bad = 0;
    auto mod_ref = [](float a, float b) -> float {
        double r = fmod((double)a, (double)b);
        if (r != 0.0 && ((r < 0.0) != (b < 0.0f))) r += (double)b;
        return (float)r;
    };
    auto mod_check = [&](float a, float b) {
        ++mod_n;
        const float got = tgp::floor_mod_f32(a, b), want = mod_ref(a, b);
        if (!((got != got && want != want) || bits(got) == bits(want))) {
            if (mod_bad < 8) printf("mod(%a, %a) = %a, want %a\n", a, b, got, want);
            ++mod_bad;
        }
    };
    for (int i = 0; i < 8000000; ++i) {
        float a, b;
        switch (i % 5) {
        case 0: a = (float)(u01(rng) * 8 - 4); b = (float)(u01(rng) * 4 - 2); break;
        case 1: a = (float)((u01(rng) - 0.5) * exp(u01(rng) * 60 - 30)); b = (float)((u01(rng) - 0.5) * exp(u01(rng) * 60 - 30)); break;
        case 2: b = (float)((u01(rng) - 0.5) * 4); a = b * (float)rint(u01(rng) * 2e7 - 1e7) * (float)(1 + (u01(rng) - 0.5) * 1e-6); break;
        case 3: b = (float)((u01(rng) - 0.5) * 4); a = (float)(rint(u01(rng) * 40 - 20)) * b; break;  // exact multiples
        default: a = (float)((u01(rng) - 0.5) * 1e-38); b = (float)((u01(rng) - 0.5) * 4); break;     // subnormal remainders
        }
        if (b != 0.0f) mod_check(a, b);
    }
    for (float a : sv)
        for (float b : sv)
            if (b != 0.0f) mod_check(a, b);
    printf("mod     %9ld cases, %ld differ from the exact floored remainder rounded once\n", mod_n, mod_bad);
    fails += mod_bad ? 1 : 0;

    // sstep, sstepp, len, lerp
    Stat s1{"sstep"}, s2{"sstepp"}, ls{"len"}, lr{"lerp"};
    for (int i = 0; i < 4000000; ++i) {
        const float x = (float)((u01(rng) - 0.5) * (i % 2 ? 6.0 : 1e3));
        const double xd = x;
        s1.add(tgp::sstep_f32(x), xd * xd * (3.0 - 2.0 * xd), 2.5, x);
        s2.add(tgp::sstepp_f32(x), xd * xd * xd * (xd * (6.0 * xd - 15.0) + 10.0), 5.0, x);
        const float y = (float)((u01(rng) - 0.5) * exp(u01(rng) * 40 - 20));
        const float x2 = (float)((u01(rng) - 0.5) * exp(u01(rng) * 40 - 20));
        ls.add(tgp::len_f32(x2, y), hypot((double)x2, (double)y), 1.5, x2, y);
        const float a = (float)((u01(rng) - 0.5) * 4), b = (float)((u01(rng) - 0.5) * 4);
        const float c = (float)((u01(rng) - 0.5) * (i % 3 ? 3.0 : 1e-3));
        const double fz = (double)c - floor((double)c);
        const double want = (double)a + ((double)b - (double)a) * fz;
        if (want != 0.0) lr.add(tgp::lerp_f32(a, b, c), want, 1.5, a, b, c);
    }
    // non-finite operands: the class of the formula's FP64 value
    const float nf[] = {INFINITY, -INFINITY, NAN, 0.0f, -0.0f, 0.5f, -1.5f, 3.0e38f, -3.0e38f};
    for (float a : nf) {
        const double ad = a;
        s1.add(tgp::sstep_f32(a), ad * ad * (3.0 - 2.0 * ad), 2.5, a);
        s2.add(tgp::sstepp_f32(a), ad * ad * ad * (ad * (6.0 * ad - 15.0) + 10.0), 5.0, a);
        for (float b : nf) {
            const double bd = b;
            ls.add(tgp::len_f32(a, b), isnan(ad) || isnan(bd) ? NAN : hypot(ad, bd), 1.5, a, b);
            for (float c : nf) {
                const double cd = c, fz = cd - floor(cd);
                const double want = ad + (bd - ad) * fz;
                if (want != 0.0 || !isfinite(want)) lr.add(tgp::lerp_f32(a, b, c), want, 1.5, a, b, c);
            }
        }
    }
    for (float big : {3.0e38f, 1e-40f, 0.0f})
        ls.add(tgp::len_f32(big, big), hypot((double)big, (double)big), 1.5, big, big);
    if (!isinf(tgp::len_f32(INFINITY, NAN)) && !isnan(tgp::len_f32(INFINITY, NAN))) ++fails;
    if (!isnan(tgp::len_f32(NAN, INFINITY)) || !isinf(tgp::len_f32(-INFINITY, 1.0f))) {
        printf("len special values\n");
        ++fails;
    }

    for (const Stat *s : {&ss, &cs, &ts, &ps, &s1, &s2, &ls, &lr}) fails += s->report();
    printf(fails ? "FAIL\n" : "OK\n");
    return fails ? 1 : 0;
}
