// Host check of the FP64-carried pow (pow_fp64.h, the same source the device
// interpreter compiles): C99 special cases bit for bit against the C
// library's powf, and random operands against the C library's FP64 pow
// rounded once to FP32 (within 1 ulp, equal in nearly every case).
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <random>
#include <vector>

#include "pow_fp64.h"

static uint32_t bits(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

// distance in ulps between two finite floats of the same sign (or zero)
static int64_t ulps(float a, float b) {
    int32_t ia, ib;
    memcpy(&ia, &a, 4);
    memcpy(&ib, &b, 4);
    if (ia < 0) ia = (int32_t)0x80000000 - ia;
    if (ib < 0) ib = (int32_t)0x80000000 - ib;
    return ia > ib ? (int64_t)ia - ib : (int64_t)ib - ia;
}

int main() {
    int bad = 0;
    // special values crossed with each other
    const float sv[] = {0.0f, -0.0f, 1.0f, -1.0f, 0.5f, -0.5f, 2.0f, -2.0f, 3.0f, -3.0f, 2.5f, -2.5f,
                        INFINITY, -INFINITY, NAN, 16777216.0f, -16777216.0f, 16777217.0f, 1e-45f, -1e-45f,
                        3.4e38f, -3.4e38f, 1.0000001f, 0.99999994f, 127.0f, -149.0f, 150.0f, -150.5f};
    for (float x : sv)
        for (float y : sv) {
            const float got = tgp::pow_fp64(x, y), want = powf(x, y);
            const bool ok = (got != got && want != want) || bits(got) == bits(want) ||
                            (isfinite(want) && want != 0.0f && ulps(got, want) <= 1);
            if (!ok) {
                printf("special pow(%a, %a) = %a, libm %a\n", x, y, got, want);
                ++bad;
            }
        }
    // random operands in the ranges GP programs produce
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> u(0.0, 1.0);
    int64_t n = 0, exact = 0, worst = 0;
    for (int i = 0; i < 4000000; ++i) {
        float x, y;
        switch (i % 4) {
        case 0:  // the grid range and a little beyond
            x = (float)(u(rng) * 4.0 - 2.0);
            y = (float)(u(rng) * 8.0 - 4.0);
            break;
        case 1:  // wide magnitudes
            x = (float)exp(u(rng) * 60.0 - 30.0);
            y = (float)(u(rng) * 20.0 - 10.0);
            break;
        case 2:  // bases near 1 with large exponents
            x = (float)(1.0 + (u(rng) - 0.5) * 1e-3);
            y = (float)((u(rng) - 0.5) * 2e5);
            break;
        default:  // negative bases with integer exponents
            x = (float)(-(u(rng) * 10.0));
            y = (float)(int)(u(rng) * 40.0 - 20.0);
            break;
        }
        const float got = tgp::pow_fp64(x, y);
        const float want = (float)pow((double)x, (double)y);
        if (want != want) {
            if (got == got) {
                printf("pow(%a, %a) = %a, want NaN\n", x, y, got);
                ++bad;
            }
            continue;
        }
        ++n;
        if (bits(got) == bits(want)) {
            ++exact;
            continue;
        }
        const int64_t d = (isinf(want) || isinf(got)) ? 1 << 30 : ulps(got, want);
        if (d > worst) worst = d;
        if (d > 1) {
            printf("pow(%a, %a) = %a, libm FP64 rounded %a (%lld ulp)\n", x, y, got, want, (long long)d);
            ++bad;
        }
    }
    printf("random: %lld cases, %lld bit-equal to the once-rounded FP64 pow, worst %lld ulp\n", (long long)n,
           (long long)exact, (long long)worst);
    if (n - exact > n / 100000) {
        printf("too many 1-ulp differences\n");
        ++bad;
    }
    printf(bad ? "FAIL\n" : "OK\n");
    return bad ? 1 : 0;
}
