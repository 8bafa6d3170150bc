// Diagnostics reduction primitives (af_diag.hip): the 11 values are 5 sums
// (4 conservative totals, entropy), 2 minima (rho, p), 2 maxima (|u| + c, c) and 2
// more sums (vorticity integral, enstrophy).
#pragma once
#include <hip/hip_runtime.h>

#include "af_internal.h"
#include "af_math.h"

namespace af {

// Tensor Simpson weights of the nine Q2 nodes of a cell summed over the cells that
// share a node: vertex 4 x 1/36, edge midpoint 2 x 4/36, centre 16/36.
constexpr double kWNodeV = 1.0 / 9.0, kWNodeE = 2.0 / 9.0, kWNodeC = 4.0 / 9.0;

__device__ __forceinline__ void diag_init(double v[kDiagVals]) {
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = 0.0;
    v[5] = v[6] = 1e300;
    v[7] = v[8] = 0.0;
    v[9] = v[10] = 0.0;
}

__device__ __forceinline__ void diag_combine(double* a, const double* b) {
#pragma unroll
    for (int k = 0; k < 5; ++k) a[k] += b[k];
    a[5] = fmin(a[5], b[5]);
    a[6] = fmin(a[6], b[6]);
    a[7] = fmax(a[7], b[7]);
    a[8] = fmax(a[8], b[8]);
    a[9] += b[9];
    a[10] += b[10];
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
    v[4] -= w * r * (log_pos(p) - gamma * log_pos(r));
    const double gp = gamma * p, cs = gp * rsqrt(gp * r);   // sqrt(gamma p / rho)
    v[5] = fmin(v[5], r);
    v[6] = fmin(v[6], p);
    v[7] = fmax(v[7], sqrt(u * u + vv * vv) + cs);
    v[8] = fmax(v[8], cs);
}

// Vorticity of a cell's Q2 velocity (nodal u[a][b], v[a][b]; a along x, b along y, on
// the nodes -1, 0, 1 of the cell's reference square) at the 3x3 Gauss-Legendre points:
// adds sum_pq w_p w_q om_pq to v[9] and sum_pq w_p w_q om_pq^2 to v[10], where
// om = (h / 2) omega.  Then int omega dA = v[9] h / 2 and int omega^2 dA = v[10]
// (the rule is exact for both).
__device__ __forceinline__ void diag_vorticity(double v[kDiagVals], const double u[3][3], const double w[3][3]) {
    constexpr double g = 0.77459666924148337704;   // sqrt(3/5)
    constexpr double gs[3] = {-g, 0.0, g}, gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    double L[3][3], dL[3][3];   // [gauss point][node]
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const double t = gs[p];
        L[p][0] = 0.5 * t * (t - 1.0); L[p][1] = 1.0 - t * t; L[p][2] = 0.5 * t * (t + 1.0);
        dL[p][0] = t - 0.5;            dL[p][1] = -2.0 * t;   dL[p][2] = t + 0.5;
    }
    // dv/dxi contracted in x first, du/deta in y first
    double vx[3][3], uy[3][3];   // vx[p][b], uy[a][q]
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            vx[p][b] = dL[p][0] * w[0][b] + dL[p][1] * w[1][b] + dL[p][2] * w[2][b];
            uy[b][p] = dL[p][0] * u[b][0] + dL[p][1] * u[b][1] + dL[p][2] * u[b][2];
        }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double dvdx = L[q][0] * vx[p][0] + L[q][1] * vx[p][1] + L[q][2] * vx[p][2];
            const double dudy = L[p][0] * uy[0][q] + L[p][1] * uy[1][q] + L[p][2] * uy[2][q];
            const double om = dvdx - dudy, wt = gw[p] * gw[q];
            v[9] += wt * om;
            v[10] += wt * om * om;
        }
}

}  // namespace af
