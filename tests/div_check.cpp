// Host check of the multiply-shift division (div_magic.h): every divisor of
// a set of awkward and random ones against exact division, on the edges of
// the 31-bit range and on random dividends.
#include <stdint.h>
#include <stdio.h>

#include <random>
#include <vector>

#include "div_magic.h"

int main() {
    std::vector<uint32_t> ds = {1, 2, 3, 5, 6, 7, 31, 32, 33, 64, 100, 255, 256, 257, 1000, 1023, 1024, 1025,
                                4095, 4096, 4097, 65535, 65536, 65537, 1000003, (1u << 30) - 1, 1u << 30,
                                (1u << 30) + 1, 0x7fffffffu};
    std::mt19937_64 rng(7);
    for (int i = 0; i < 200; ++i) ds.push_back(1 + (uint32_t)(rng() % 0x7fffffffu));
    int bad = 0;
    int64_t checked = 0;
    for (uint32_t d : ds) {
        uint32_t m, s;
        tgp::div_magic(d, &m, &s);
        auto check = [&](uint32_t n) {
            ++checked;
            if (tgp::div_by_magic(n, m, s) != n / d) {
                if (bad < 10) printf("n %u d %u: %u != %u\n", n, d, tgp::div_by_magic(n, m, s), n / d);
                ++bad;
            }
        };
        for (uint32_t n = 0; n < 4096; ++n) check(n);
        for (uint32_t n = 0x7fffffffu - 4096; n < 0x7fffffffu; ++n) check(n);
        check(0x7fffffffu);
        for (uint64_t k = 1; k * d < 0x80000000ull && k < 100000; k = k * 3 + 1) {
            check((uint32_t)(k * d - 1));
            check((uint32_t)(k * d));
            if (k * d + 1 < 0x80000000ull) check((uint32_t)(k * d + 1));
        }
        for (int i = 0; i < 20000; ++i) check((uint32_t)(rng() & 0x7fffffffu));
    }
    printf("%lld quotients checked, %d wrong\n", (long long)checked, bad);
    printf(bad ? "FAIL\n" : "OK\n");
    return bad ? 1 : 0;
}
