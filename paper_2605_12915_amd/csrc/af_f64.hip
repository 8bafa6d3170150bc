// FP64 RB-TAI Active Flux step for gfx950: multi-kernel reference path.
//
// Four launches per step, one thread per cell, periodic gathers from global
// memory (L2-served):
//   k_centre   recovered centre node W^C (eq. center-node)
//   k_incr     acoustic increments at V, Ev, Eh, C for tau = dt/2 and dt (App. D)
//   k_points   transported point update of V, Ev, Eh at n+1/2 and n+1 (Sec. 6.1)
//   k_update   space-time Simpson fluxes and the average update (eq. af-average-update)
// This path stores the intermediates (W^C, 24 increment planes, 12 half-time
// planes) in the context's scratch; the fused kernel in af_fused.hip keeps them
// on chip.
// The foot-centred exact update (AF_SCHEME_FC) runs here too: k_centre, then
// k_fc_points in place of k_incr and k_points, then k_update.
#include <hip/hip_runtime.h>

#include "af_footcentred.h"
#include "af_internal.h"
#include "af_kernels.h"

namespace af {

struct GAcc64 {
    const double* s[16];
    const double* C;      // 4 planes
    int nx, ny;
    __device__ __forceinline__ size_t idx(int i, int j) const {
        i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
        j = (j < 0) ? j + ny : (j >= ny ? j - ny : j);
        return (size_t)j * nx + i;
    }
    __device__ __forceinline__ Prim<double> node(int fam, int i, int j) const {
        size_t k = idx(i, j);
        if (fam == F_C) {
            size_t N = (size_t)nx * ny;
            return {C[k], C[N + k], C[2 * N + k], C[3 * N + k]};
        }
        const int b = 4 + 4 * fam;
        return {s[b][k], s[b + 1][k], s[b + 2][k], s[b + 3][k]};
    }
};

struct GInc64 {
    const double* d;      // 12 planes for one tau: [fam][var]
    int nx, ny;
    __device__ __forceinline__ double inc(int fam, int i, int j, int var) const {
        i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
        j = (j < 0) ? j + ny : (j >= ny ? j - ny : j);
        return d[(size_t)(fam * 3 + var) * nx * ny + (size_t)j * nx + i];
    }
};

__global__ void __launch_bounds__(256) k_centre(StatePtrs<double> in, double* C, int nx, int ny, double gamma,
                                                unsigned* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    GAcc64 A{{}, nullptr, nx, ny};
#pragma unroll
    for (int k = 0; k < 16; ++k) A.s[k] = in.p[k];
    const size_t c = (size_t)j * nx + i;
    double Ub[4] = {in.p[0][c], in.p[1][c], in.p[2][c], in.p[3][c]};
    Prim<double> w = recover_centre(Ub, A.node(F_V, i, j), A.node(F_V, i + 1, j), A.node(F_V, i, j + 1),
                                    A.node(F_V, i + 1, j + 1), A.node(F_EH, i, j), A.node(F_EH, i, j + 1),
                                    A.node(F_EV, i, j), A.node(F_EV, i + 1, j), gamma);
    const size_t N = (size_t)nx * ny;
    C[c] = w.r;
    C[N + c] = w.u;
    C[2 * N + c] = w.v;
    C[3 * N + c] = w.p;
    if (!(w.r > 0.0) || !(w.p > 0.0)) atomicOr(status, (unsigned)SB_NONPHYS);
}

__global__ void __launch_bounds__(256) k_incr(StatePtrs<double> in, const double* C, double* inc, int nx, int ny,
                                              double gamma, double lam0, double lam1, unsigned* status) {
    const PolAbs<double> pol{gamma, 1.0 / (gamma - 1.0)};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    GAcc64 A{{}, C, nx, ny};
#pragma unroll
    for (int k = 0; k < 16; ++k) A.s[k] = in.p[k];
    unsigned st = 0;
    double d[2][3];
    const size_t N = (size_t)nx * ny, c = (size_t)j * nx + i;
    node_increments<F_V>(A, i, j, pol, lam0, lam1, d, st);
    for (int t = 0; t < 2; ++t)
        for (int v = 0; v < 3; ++v) inc[(size_t)(t * 12 + 0 * 3 + v) * N + c] = d[t][v];
    node_increments<F_EV>(A, i, j, pol, lam0, lam1, d, st);
    for (int t = 0; t < 2; ++t)
        for (int v = 0; v < 3; ++v) inc[(size_t)(t * 12 + 1 * 3 + v) * N + c] = d[t][v];
    node_increments<F_EH>(A, i, j, pol, lam0, lam1, d, st);
    for (int t = 0; t < 2; ++t)
        for (int v = 0; v < 3; ++v) inc[(size_t)(t * 12 + 2 * 3 + v) * N + c] = d[t][v];
    node_increments<F_C>(A, i, j, pol, lam0, lam1, d, st);
    for (int t = 0; t < 2; ++t)
        for (int v = 0; v < 3; ++v) inc[(size_t)(t * 12 + 3 * 3 + v) * N + c] = d[t][v];
    if (st) atomicOr(status, st);
}

template <int SCHEME>
__global__ void __launch_bounds__(256) k_points(StatePtrs<double> in, const double* C, const double* inc,
                                                double* half, StatePtrs<double> out, int nx, int ny,
                                                double gamma, double lam0, double lam1, unsigned* status) {
    const PolAbs<double> pol{gamma, 1.0 / (gamma - 1.0)};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    GAcc64 A{{}, C, nx, ny};
#pragma unroll
    for (int k = 0; k < 16; ++k) A.s[k] = in.p[k];
    const size_t N = (size_t)nx * ny, c = (size_t)j * nx + i;
    unsigned st = 0;
    for (int t = 0; t < 2; ++t) {
        GInc64 D{inc + (size_t)t * 12 * N, nx, ny};
        const double lam = t ? lam1 : lam0;
        Prim<double> w[3];
        w[0] = point_update<F_V, SCHEME>(A, D, i, j, pol, lam, st);
        w[1] = point_update<F_EV, SCHEME>(A, D, i, j, pol, lam, st);
        w[2] = point_update<F_EH, SCHEME>(A, D, i, j, pol, lam, st);
        for (int f = 0; f < 3; ++f) {
            double vals[4] = {w[f].r, w[f].u, w[f].v, w[f].p};
            for (int k = 0; k < 4; ++k) {
                if (t == 0) half[(size_t)(4 * f + k) * N + c] = vals[k];
                else out.p[4 + 4 * f + k][c] = vals[k];
            }
        }
    }
    if (st) atomicOr(status, st);
}

// Time-Simpson combination of the flux at one node: (F(W^0) + 4 F(W^1/2) + F(W^1)) / 6.
__device__ __forceinline__ void tflux(const Prim<double>& a, const Prim<double>& b, const Prim<double>& c,
                                      double gm1inv, bool xdir, double out[4]) {
    double Fa[4], Fb[4], Fc[4];
    if (xdir) { flux_x(a, gm1inv, Fa); flux_x(b, gm1inv, Fb); flux_x(c, gm1inv, Fc); }
    else { flux_y(a, gm1inv, Fa); flux_y(b, gm1inv, Fb); flux_y(c, gm1inv, Fc); }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = (Fa[k] + 4.0 * Fb[k] + Fc[k]) * (1.0 / 6.0);
}

__global__ void __launch_bounds__(256) k_update(StatePtrs<double> in, const double* half, StatePtrs<double> out,
                                                int nx, int ny, double gamma, double lam) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t N = (size_t)nx * ny;
    auto id = [&](int a, int b) -> size_t {
        a = a >= nx ? a - nx : a;
        b = b >= ny ? b - ny : b;
        return (size_t)b * nx + a;
    };
    auto pt = [&](int lvl, int fam, int a, int b) -> Prim<double> {
        size_t k = id(a, b);
        if (lvl == 0) { const int q = 4 + 4 * fam; return {in.p[q][k], in.p[q + 1][k], in.p[q + 2][k], in.p[q + 3][k]}; }
        if (lvl == 1) { const double* h = half + (size_t)(4 * fam) * N; return {h[k], h[N + k], h[2 * N + k], h[3 * N + k]}; }
        const int q = 4 + 4 * fam;
        return {out.p[q][k], out.p[q + 1][k], out.p[q + 2][k], out.p[q + 3][k]};
    };
    const double gm1inv = 1.0 / (gamma - 1.0);
    double FV00[4], FV01[4], FV10[4], FV11[4], FE0[4], FE1[4];
    double GV00[4], GV10[4], GV01[4], GV11[4], GE0[4], GE1[4];
    tflux(pt(0, F_V, i, j), pt(1, F_V, i, j), pt(2, F_V, i, j), gm1inv, true, FV00);
    tflux(pt(0, F_V, i, j), pt(1, F_V, i, j), pt(2, F_V, i, j), gm1inv, false, GV00);
    tflux(pt(0, F_V, i, j + 1), pt(1, F_V, i, j + 1), pt(2, F_V, i, j + 1), gm1inv, true, FV01);
    tflux(pt(0, F_V, i, j + 1), pt(1, F_V, i, j + 1), pt(2, F_V, i, j + 1), gm1inv, false, GV01);
    tflux(pt(0, F_V, i + 1, j), pt(1, F_V, i + 1, j), pt(2, F_V, i + 1, j), gm1inv, true, FV10);
    tflux(pt(0, F_V, i + 1, j), pt(1, F_V, i + 1, j), pt(2, F_V, i + 1, j), gm1inv, false, GV10);
    tflux(pt(0, F_V, i + 1, j + 1), pt(1, F_V, i + 1, j + 1), pt(2, F_V, i + 1, j + 1), gm1inv, true, FV11);
    tflux(pt(0, F_V, i + 1, j + 1), pt(1, F_V, i + 1, j + 1), pt(2, F_V, i + 1, j + 1), gm1inv, false, GV11);
    tflux(pt(0, F_EV, i, j), pt(1, F_EV, i, j), pt(2, F_EV, i, j), gm1inv, true, FE0);
    tflux(pt(0, F_EV, i + 1, j), pt(1, F_EV, i + 1, j), pt(2, F_EV, i + 1, j), gm1inv, true, FE1);
    tflux(pt(0, F_EH, i, j), pt(1, F_EH, i, j), pt(2, F_EH, i, j), gm1inv, false, GE0);
    tflux(pt(0, F_EH, i, j + 1), pt(1, F_EH, i, j + 1), pt(2, F_EH, i, j + 1), gm1inv, false, GE1);
    const size_t c = (size_t)j * nx + i;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double Fl = (FV00[k] + 4.0 * FE0[k] + FV01[k]) * (1.0 / 6.0);
        double Fr = (FV10[k] + 4.0 * FE1[k] + FV11[k]) * (1.0 / 6.0);
        double Gb = (GV00[k] + 4.0 * GE0[k] + GV10[k]) * (1.0 / 6.0);
        double Gt = (GV01[k] + 4.0 * GE1[k] + GV11[k]) * (1.0 / 6.0);
        out.p[k][c] = in.p[k][c] - lam * ((Fr - Fl) + (Gt - Gb));
    }
}

// Foot-centred exact point update (af_footcentred.h) of every target for both
// durations: item e is duration e / 3N, family (e / N) mod 3, cell e mod N, so that
// consecutive lanes take consecutive cells of one family and duration.  Registers
// bounded for two workgroups per CU (2 waves per SIMD; 21% faster than the unbounded
// allocation at one, 4x slower at four waves per SIMD, where it spills).
__global__ void __launch_bounds__(256, 2) k_fc_points(StatePtrs<double> in, const double* C, double* half,
                                                   StatePtrs<double> out, int nx, int ny, double gamma, double lam0,
                                                   double lam1, unsigned* status) {
    const size_t N = (size_t)nx * ny, total = 6 * N;
    GAcc64 A{{}, C, nx, ny};
#pragma unroll
    for (int k = 0; k < 16; ++k) A.s[k] = in.p[k];
    unsigned st = 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int tau = e >= 3 * N ? 1 : 0;
        const size_t r = e - (size_t)tau * 3 * N;
        const int fam = (int)(r / N);
        const size_t c = r - (size_t)fam * N;
        const int i = (int)(c % nx), j = (int)(c / nx);
        const Prim<double> w = fc_point_update(A, fam, i, j, gamma, tau ? lam1 : lam0, st);
        double* const q[4] = {tau ? out.p[4 + 4 * fam] : half + (size_t)(4 * fam) * N,
                              tau ? out.p[5 + 4 * fam] : half + (size_t)(4 * fam + 1) * N,
                              tau ? out.p[6 + 4 * fam] : half + (size_t)(4 * fam + 2) * N,
                              tau ? out.p[7 + 4 * fam] : half + (size_t)(4 * fam + 3) * N};
        q[0][c] = w.r;
        q[1][c] = w.u;
        q[2][c] = w.v;
        q[3][c] = w.p;
    }
    if (st) atomicOr(status, st);
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
hipError_t launch_step_multi_f64(const StepArgs& a) {
    dim3 blk(64, 4), grd((a.nx + 63) / 64, (a.ny + 3) / 4);
    StatePtrs<double> in, out;
    for (int k = 0; k < 16; ++k) { in.p[k] = (double*)a.in[k]; out.p[k] = (double*)a.out[k]; }
    double* C = (double*)a.scratch;
    const size_t N = (size_t)a.nx * a.ny;
    double* inc = C + 4 * N;
    double* half = inc + 24 * N;
    const double lam1 = a.dt / a.h, lam0 = 0.5 * lam1;
    hipLaunchKernelGGL(k_centre, grd, blk, 0, a.stream, in, C, a.nx, a.ny, a.gamma, a.status);
    hipLaunchKernelGGL(k_incr, grd, blk, 0, a.stream, in, C, inc, a.nx, a.ny, a.gamma, lam0, lam1, a.status);
    if (a.ev_begin) (void)hipEventRecord(a.ev_begin, a.stream);
    if (a.scheme == 0)
        hipLaunchKernelGGL(k_points<0>, grd, blk, 0, a.stream, in, C, inc, half, out, a.nx, a.ny, a.gamma, lam0, lam1,
                           a.status);
    else
        hipLaunchKernelGGL(k_points<1>, grd, blk, 0, a.stream, in, C, inc, half, out, a.nx, a.ny, a.gamma, lam0, lam1,
                           a.status);
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    hipLaunchKernelGGL(k_update, grd, blk, 0, a.stream, in, half, out, a.nx, a.ny, a.gamma, lam1);
    return hipGetLastError();
}

size_t scratch_bytes_multi_f64(int nx, int ny) { return (size_t)nx * ny * (4 + 24 + 12) * sizeof(double); }

hipError_t launch_step_fc_f64(const StepArgs& a) {
    dim3 blk(64, 4), grd((a.nx + 63) / 64, (a.ny + 3) / 4);
    StatePtrs<double> in, out;
    for (int k = 0; k < 16; ++k) { in.p[k] = (double*)a.in[k]; out.p[k] = (double*)a.out[k]; }
    double* C = (double*)a.scratch;
    const size_t N = (size_t)a.nx * a.ny;
    double* half = C + 4 * N;
    const double lam1 = a.dt / a.h, lam0 = 0.5 * lam1;
    hipLaunchKernelGGL(k_centre, grd, blk, 0, a.stream, in, C, a.nx, a.ny, a.gamma, a.status);
    const size_t items = 6 * N, blocks = (items + 255) / 256;
    if (a.ev_begin) (void)hipEventRecord(a.ev_begin, a.stream);
    hipLaunchKernelGGL(k_fc_points, dim3((unsigned)(blocks < (1u << 20) ? blocks : (1u << 20))), dim3(256), 0,
                       a.stream, in, C, half, out, a.nx, a.ny, a.gamma, lam0, lam1, a.status);
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    hipLaunchKernelGGL(k_update, grd, blk, 0, a.stream, in, half, out, a.nx, a.ny, a.gamma, lam1);
    return hipGetLastError();
}

size_t scratch_bytes_fc_f64(int nx, int ny) { return (size_t)nx * ny * (4 + 12) * sizeof(double); }

}  // namespace af
