// Host build of af::log_pos (csrc/af_math.h) against the host's log: largest distance in
// units in the last place over a sweep of arguments (every binade of the normal range at
// 4096 mantissas each, both neighbourhoods of 1, the subnormal range, and seeded random
// doubles).  Prints {"max_ulp": ..., "count": ...}.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "af_math.h"

static int64_t ordered(double v) {
    int64_t b;
    std::memcpy(&b, &v, 8);
    return b < 0 ? INT64_MIN - b : b;
}

int main() {
    double worst = 0.0, worst_x = 0.0;
    long count = 0;
    auto check = [&](double x) {
        const double got = af::log_pos(x), want = std::log(x);
        if (want == 0.0) {
            if (got != 0.0 && std::fabs(got) > 1e-300) { worst = 1e9; worst_x = x; }
            ++count;
            return;
        }
        const double d = (double)std::llabs(ordered(got) - ordered(want));
        if (d > worst) { worst = d; worst_x = x; }
        ++count;
    };
    for (int e = -1022; e <= 1023; ++e)
        for (int k = 0; k < 4096; ++k) check(std::ldexp(1.0 + k / 4096.0, e));
    for (int k = 1; k <= 200000; ++k) {
        check(1.0 + k * 1e-12);
        check(1.0 - k * 1e-12);
        check(1.0 + k * 1e-6);
        check(1.0 - k * 1e-6);
    }
    for (int k = 1; k < 100000; ++k) check(std::ldexp((double)k, -1074));
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> mant(1.0, 2.0);
    std::uniform_int_distribution<int> ex(-1000, 1000);
    for (int k = 0; k < 2000000; ++k) check(std::ldexp(mant(rng), ex(rng)));
    std::printf("{\"max_ulp\": %.0f, \"worst_x\": %.17g, \"count\": %ld}\n", worst, worst_x, count);
    return 0;
}
