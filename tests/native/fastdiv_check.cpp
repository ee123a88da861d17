// Host check of the invariant-divisor division and the local-index helper
// used by the device code: every result is compared with plain C++ integer
// division. Built with hipcc as host code only; prints "ok" or the first
// mismatch.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "common.h"

using corr::Box;
using corr::FastDiv;

static int check_div(uint32_t d, uint32_t n) {
    const FastDiv f(d);
    if (f.div(n) != n / d) {
        std::printf("mismatch: %u / %u gave %u, expected %u\n", n, d, f.div(n), n / d);
        return 1;
    }
    return 0;
}

int main() {
    std::mt19937_64 rng(12345);
    const uint32_t top = 0x7fffffffu;
    // every divisor up to 4096 against edge and random numerators
    for (uint32_t d = 1; d <= 4096; ++d) {
        const uint32_t edge[] = {0, 1, d - 1, d, d + 1, 2 * d - 1, 2 * d, top, top - 1, top - d, top / d * d,
                                 top / d * d - 1};
        for (uint32_t n : edge)
            if (n <= top && check_div(d, n)) return 1;
        for (int r = 0; r < 2000; ++r)
            if (check_div(d, (uint32_t)(rng() & top))) return 1;
    }
    // every numerator below 2^20 for a few divisors, and random large divisors
    const uint32_t ds[] = {3, 7, 80, 250, 352, 640, 704, 1000, 2560, 65535, 65536, 65537};
    for (uint32_t d : ds)
        for (uint32_t n = 0; n < (1u << 20); ++n)
            if (check_div(d, n)) return 1;
    for (int r = 0; r < 200000; ++r) {
        const uint32_t d = 1 + (uint32_t)(rng() % top);
        if (check_div(d, (uint32_t)(rng() & top)) || check_div(d, d) || check_div(d, d - 1)) return 1;
    }
    // local indices against Box::local on ragged boxes of a few grids
    const int grids[][3] = {{16, 8, 4}, {80, 32, 20}, {352, 256, 20}, {128, 128, 32}, {7, 5, 3}};
    for (auto& g : grids) {
        const FastDiv fx((uint32_t)g[0]), fy((uint32_t)g[1]);
        for (int t = 0; t < 50; ++t) {
            Box b{};
            b.nx = g[0];
            b.ny = g[1];
            b.x0 = (int)(rng() % g[0]);
            b.y0 = (int)(rng() % g[1]);
            b.z0 = (int)(rng() % g[2]);
            b.dx = 1 + (int)(rng() % (g[0] - b.x0));
            b.dy = 1 + (int)(rng() % (g[1] - b.y0));
            b.dz = 1 + (int)(rng() % (g[2] - b.z0));
            for (int p = 0; p < g[0] * g[1] * g[2]; ++p)
                if (corr::box_local_fast(b, fx, fy, p) != b.local(p)) {
                    std::printf("local index mismatch at p = %d\n", p);
                    return 1;
                }
        }
    }
    std::printf("ok\n");
    return 0;
}
