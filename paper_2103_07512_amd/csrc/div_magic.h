// div_magic.h -- division of 31-bit unsigned integers by an invariant
// divisor with one high multiply and a shift (Granlund & Montgomery,
// "Division by invariant integers using multiplication", PLDI 1994,
// Theorem 4.2 with N = 31): for d >= 2, l = ceil(log2 d) and
// m = ceil(2^(31 + l) / d) < 2^32, floor(n / d) = floor(n m / 2^(31 + l))
// = (high 32 bits of n m) >> (l - 1) for every 0 <= n < 2^31.  d = 1 is
// marked by m = 0 (the quotient is n).
#pragma once

#include <stdint.h>

#ifndef TGP_HD
#ifdef __HIPCC__
#define TGP_HD __host__ __device__
#else
#define TGP_HD
#endif
#endif

namespace tgp {

inline void div_magic(uint32_t d, uint32_t *m, uint32_t *shift) {
    if (d <= 1) {
        *m = 0;
        *shift = 0;
        return;
    }
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    *m = (uint32_t)(((1ull << (31 + l)) + d - 1) / d);
    *shift = l - 1;
}

// The quotient as the device computes it (also compiled for the host tests).
TGP_HD inline uint32_t div_by_magic(uint32_t n, uint32_t m, uint32_t shift) {
    return m ? (uint32_t)(((uint64_t)n * m) >> 32) >> shift : n;
}

}  // namespace tgp
