// Diagnostics reduction primitives (af_diag.hip): the 9 values are 5 sums
// (4 conservative totals, entropy), 2 minima (rho, p) and 2 maxima (|u| + c, c).
#pragma once
#include <hip/hip_runtime.h>

#include "af_internal.h"

namespace af {

// Tensor Simpson weights of the nine Q2 nodes of a cell summed over the cells that
// share a node: vertex 4 x 1/36, edge midpoint 2 x 4/36, centre 16/36.
constexpr double kWNodeV = 1.0 / 9.0, kWNodeE = 2.0 / 9.0, kWNodeC = 4.0 / 9.0;

__device__ __forceinline__ void diag_init(double v[kDiagVals]) {
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = 0.0;
    v[5] = v[6] = 1e300;
    v[7] = v[8] = 0.0;
}

__device__ __forceinline__ void diag_combine(double* a, const double* b) {
#pragma unroll
    for (int k = 0; k < 5; ++k) a[k] += b[k];
    a[5] = fmin(a[5], b[5]);
    a[6] = fmin(a[6], b[6]);
    a[7] = fmax(a[7], b[7]);
    a[8] = fmax(a[8], b[8]);
}

// Lane 0 of each 64-wide wavefront ends with the wavefront's reduction.
__device__ __forceinline__ void diag_wave_reduce(double v[kDiagVals]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o[kDiagVals];
#pragma unroll
        for (int k = 0; k < kDiagVals; ++k) o[k] = __shfl_down(v[k], off, 64);
        diag_combine(v, o);
    }
}

// Diagnostics of one node given as absolute FP64 (rho, u, v, p): entropy density
// weighted by w, minima and maxima.
__device__ __forceinline__ void diag_node(double v[kDiagVals], double w, double r, double u, double vv, double p,
                                          double gamma) {
    v[4] -= w * r * (log(p) - gamma * log(r));
    const double cs = sqrt(gamma * p / r);
    v[5] = fmin(v[5], r);
    v[6] = fmin(v[6], p);
    v[7] = fmax(v[7], sqrt(u * u + vv * vv) + cs);
    v[8] = fmax(v[8], cs);
}

}  // namespace af
