// Natural logarithm of a positive double, for the diagnostics' entropy density (eight
// logarithms per cell).  x = m 2^e with m in [1/sqrt(2), sqrt(2)), so that
//   log x = e log 2 + 2 atanh(t),   t = (m - 1) / (m + 1),   |t| <= 3 - 2 sqrt(2) < 0.1716,
// with atanh summed by its Taylor series t + t^3/3 + t^5/5 + ... through the t^21 term
// (the first term left out is below 1e-18 of the sum).  m - 1 is exact and t carries two
// roundings: over 11 million arguments from every binade, both sides of 1 and the
// subnormals, the result lies within 2 ulp of the host's log (tests/log_host.cpp).  About
// 30 instructions on gfx950 against about 100 for the device library's log.  log 0 = -inf,
// log inf = inf, and negative or NaN arguments give NaN.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#ifndef AF_HD
#define AF_HD __host__ __device__ __forceinline__
#endif

namespace af {

AF_HD double log_pos(double x) {
    if (!(x > 0.0 && x < HUGE_VAL)) return x == 0.0 ? -HUGE_VAL : (x == HUGE_VAL ? x : __builtin_nan(""));
    int e;
    double m = frexp(x, &e);   // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double t = (m - 1.0) / (m + 1.0), t2 = t * t;
    double s = 1.0 / 21.0;
    s = fma(s, t2, 1.0 / 19.0);
    s = fma(s, t2, 1.0 / 17.0);
    s = fma(s, t2, 1.0 / 15.0);
    s = fma(s, t2, 1.0 / 13.0);
    s = fma(s, t2, 1.0 / 11.0);
    s = fma(s, t2, 1.0 / 9.0);
    s = fma(s, t2, 1.0 / 7.0);
    s = fma(s, t2, 1.0 / 5.0);
    s = fma(s, t2, 1.0 / 3.0);
    const double tt = 2.0 * t;   // 2 atanh(t) = 2t + 2t t^2 s
    return fma((double)e, 0.69314718055994530942, fma(tt * t2, s, tt));
}

}  // namespace af
