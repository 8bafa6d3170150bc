// Reverse-mode derivative of one FP64 RB-TAI step (transposed Sec. 6.1 dataflow).
//
// cot_n = (d step / d state_n)^T cot_np1 at fixed dt, in three kernels.  The reverse
// of a gather stencil is a scatter: every block accumulates its scattered
// contributions in an LDS window over its cells plus the reach of the stencil (LDS
// FP64 atomics), then adds the window to global memory once (one global atomic per
// window entry instead of one per contribution):
//   k_adj_fwd      forward intermediates recomputed from state_n (recovered centres
//                  W^C, node increments of both durations); zeroes the accumulation
//                  planes and starts the averages' cotangent at cot_np1's.
//   k_adj_points   average update and space-time Simpson fluxes (transposed), then
//                  for every target and duration the transposed point update (TAI:
//                  density closure, Q2 evaluation of W and of the increments at the
//                  foot, values and foot position, the two Picard stages; RB: Q2 of W
//                  at the foot, the target's own increments).  Scatters into cot_n
//                  (point planes), lambda_C and lambda_D.
//   k_adj_incr     transposed node increments (Horner in r, freezing c_K, Z_K,
//                  transposed monomial blocks and Lagrange-to-monomial transforms of
//                  every wedge), then the transposed centre recovery (prim(U_c),
//                  inverse Simpson, U(W) at the eight boundary nodes) applied to each
//                  block's own share of lambda_C; scatters into the point and average
//                  planes of cot_n.
// The floor() that locates a foot is piecewise constant: its derivative is zero
// (the usual convention; the step is continuous across faces because R_h and I_h are).
#include <hip/hip_runtime.h>

#include "af_internal.h"
#include "af_kernels.h"

namespace af {

struct AdjNodes {
    const double* s[16];
    const double* C;
    int nx, ny;
    __device__ __forceinline__ size_t idx(int i, int j) const {
        i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
        j = (j < 0) ? j + ny : (j >= ny ? j - ny : j);
        return (size_t)j * nx + i;
    }
    __device__ __forceinline__ double comp(int fam, int i, int j, int q) const {
        const size_t k = idx(i, j);
        if (fam == F_C) return C[(size_t)q * nx * ny + k];
        return s[4 + 4 * fam + q][k];
    }
    __device__ __forceinline__ Prim<double> node(int fam, int i, int j) const {
        const size_t k = idx(i, j);
        if (fam == F_C) {
            const size_t N = (size_t)nx * ny;
            return {C[k], C[N + k], C[2 * N + k], C[3 * N + k]};
        }
        const int b = 4 + 4 * fam;
        return {s[b][k], s[b + 1][k], s[b + 2][k], s[b + 3][k]};
    }
};

// Scatter target of the reverse sweep: an LDS window of NPL planes over node-cells
// [ri0, ri0 + RX) x [rj0, rj0 + RY) (unwrapped indices; the flush wraps them).
// Planes: 0..11 point values (family * 4 + (rho, u, v, p)), 12..15 recovered
// centres, 16..39 increments (tau * 12 + family * 3 + (u, v, p)).
template <int NPL, int RX, int RY>
struct LdsWin {
    double* a;
    int ri0, rj0;
    static constexpr int kRX = RX, kPlane = RX * RY;
    __device__ __forceinline__ void add(int pl, int i, int j, double v) const {
        atomicAdd(a + (pl * RY + (j - rj0)) * RX + (i - ri0), v);
    }
    // offset of node-cell (i, j) within a plane; addb adds to plane pl at that offset
    // plus a small constant one (so that every add of one cell's nodes shares a base)
    __device__ __forceinline__ int base(int i, int j) const { return (j - rj0) * RX + (i - ri0); }
    __device__ __forceinline__ void addb(int pl, int b, int off, double v) const {
        atomicAdd(a + b + (pl * kPlane + off), v);
    }
    // add g = (d rho, d u, d v, d p) to node fam of cell (i, j)
    __device__ __forceinline__ void node(int fam, int i, int j, const double g[4]) const {
        const int b = fam == F_C ? 12 : 4 * fam, o = base(i, j);
#pragma unroll
        for (int q = 0; q < 4; ++q) addb(b + q, o, 0, g[q]);
    }
    __device__ __forceinline__ void zero() const {
        for (int e = threadIdx.x; e < NPL * RX * RY; e += blockDim.x) a[e] = 0.0;
    }
};

struct PlaneList { double* p[40]; };

// The forward state of a block, staged in LDS over the node-cells of its scatter
// window with the window's plane numbering: point values (0..11), recovered centres
// (12..15), increments of both durations (16..39).
template <int RX, int RY>
struct StageWin {
    const double* a;
    int ri0, rj0;
    static constexpr int kRX = RX, kPlane = RX * RY;
    __device__ __forceinline__ int base(int i, int j) const { return (j - rj0) * RX + (i - ri0); }
    __device__ __forceinline__ double at(int pl, int b, int off) const { return a[b + (pl * kPlane + off)]; }
    __device__ __forceinline__ Prim<double> node(int fam, int b) const {
        const int pl = fam == F_C ? 12 : 4 * fam;
        return {at(pl, b, 0), at(pl + 1, b, 0), at(pl + 2, b, 0), at(pl + 3, b, 0)};
    }
};

// Add an LDS window to its global planes (periodic wrap), one atomic per nonzero entry:
// each thread takes whole node-cells of the window, wraps its global index once and
// walks the planes (so the plane pointer is the same across the wavefront).
template <int NPL, int RX, int RY>
__device__ __forceinline__ void flush_window(const LdsWin<NPL, RX, RY>& w, const PlaneList& G, int nx, int ny) {
    for (int e = threadIdx.x; e < RX * RY; e += blockDim.x) {
        int i = w.ri0 + e % RX, j = w.rj0 + e / RX;
        i = (i % nx + nx) % nx;
        j = (j % ny + ny) % ny;
        const size_t k = (size_t)j * nx + i;
#pragma unroll 8
        for (int pl = 0; pl < NPL; ++pl) {
            const double v = w.a[pl * (RX * RY) + e];
            if (v != 0.0) atomicAdd(G.p[pl] + k, v);
        }
    }
}

// Family of node [a][b] of a cell, the node-cell (dx, dy) of the cell's 2x2 block of
// node-cells that holds it, and its first plane in the scatter window (point values
// fam * 4, centre 12).
__device__ __forceinline__ constexpr int fam_of(int a, int b) {
    return (a == 1 && b == 1) ? F_C : (a == 1 ? F_EH : (b == 1 ? F_EV : F_V));
}
__device__ __forceinline__ constexpr int win_plane(int fam) { return fam == F_C ? 12 : 4 * fam; }

// Periodic index: one shift (offsets of at most one grid length) or a modulo.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int wrap_any(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ void lagr(double s, double l[3], double dl[3]) {
    l[0] = 0.5 * s * (s - 1.0);
    l[1] = 1.0 - s * s;
    l[2] = 0.5 * s * (s + 1.0);
    dl[0] = s - 0.5;
    dl[1] = -2.0 * s;
    dl[2] = s + 0.5;
}

// Flux Jacobians transposed: g += (dF/dW)^T nu, W = (rho, u, v, p).
__device__ __forceinline__ void flux_x_T(const Prim<double>& w, double gamma, const double nu[4], double g[4]) {
    const double q2 = 0.5 * (w.u * w.u + w.v * w.v);
    const double E = w.p / (gamma - 1.0) + w.r * q2;
    g[0] += nu[0] * w.u + nu[1] * w.u * w.u + nu[2] * w.u * w.v + nu[3] * w.u * q2;
    g[1] += nu[0] * w.r + nu[1] * 2.0 * w.r * w.u + nu[2] * w.r * w.v + nu[3] * (E + w.p + w.r * w.u * w.u);
    g[2] += nu[2] * w.r * w.u + nu[3] * w.r * w.u * w.v;
    g[3] += nu[1] + nu[3] * w.u * gamma / (gamma - 1.0);
}

__device__ __forceinline__ void flux_y_T(const Prim<double>& w, double gamma, const double nu[4], double g[4]) {
    const double q2 = 0.5 * (w.u * w.u + w.v * w.v);
    const double E = w.p / (gamma - 1.0) + w.r * q2;
    g[0] += nu[0] * w.v + nu[1] * w.u * w.v + nu[2] * w.v * w.v + nu[3] * w.v * q2;
    g[1] += nu[1] * w.r * w.v + nu[3] * w.r * w.u * w.v;
    g[2] += nu[0] * w.r + nu[1] * w.r * w.u + nu[2] * 2.0 * w.r * w.v + nu[3] * (E + w.p + w.r * w.v * w.v);
    g[3] += nu[2] + nu[3] * w.v * gamma / (gamma - 1.0);
}

// Transposed point update of target FAM at (i, j) for the duration tau = lam h;
// WP = the target's time-n value.  SCHEME 0: transported update (the increments are
// interpolated at the foot, the density closure uses c^2 at the foot); SCHEME 1:
// additive update (the target's own increments, c^2 frozen at the target).
// The forward value w is recomputed here and its cotangent formed from the flux
// cotangents: lw = ws * (dF/dW)^T nuF + ws * (dG/dW)^T nuG (+ extra: the cotangent
// of the new point value itself, for the full step).  The contributions to the
// target's own node (through the first foot position) are added to gself, those to
// the nodes of the two foot cells go to the window, one base offset per cell.
template <int FAM, int SCHEME, class S_, class O_>
__device__ void point_update_adj(const S_& S, const O_& O, int t, int i, int j, const Prim<double>& WP,
                                 double gamma, double lam, const double nuF[4], const double nuG[4], double ws,
                                 const double* extra, double gself[4]) {
    const double ox = FamOffset<FAM>::ox, oy = FamOffset<FAM>::oy;
    constexpr int RX = O_::kRX;
    static_assert(S_::kRX == O_::kRX && S_::kPlane == O_::kPlane, "staged state and window share a layout");
    unsigned st = 0;
    // ---- forward recomputation ----
    int cx1, cy1, cx2, cy2;
    double xi1, eta1, xi2, eta2;
    locate(ox - lam * WP.u, ox, cx1, xi1, st);
    locate(oy - lam * WP.v, oy, cy1, eta1, st);
    double lx1[3], dlx1[3], ly1[3], dly1[3];
    lagr(xi1, lx1, dlx1);
    lagr(eta1, ly1, dly1);
    double u1 = 0.0, v1 = 0.0, du1x = 0.0, du1y = 0.0, dv1x = 0.0, dv1y = 0.0;
    const int wb1 = O.base(i + cx1, j + cy1);
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int f = fam_of(a, b), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
                const double nu_ = S.at(win_plane(f) + 1, wb1, off), nv_ = S.at(win_plane(f) + 2, wb1, off);
                u1 += lx1[a] * ly1[b] * nu_;
                v1 += lx1[a] * ly1[b] * nv_;
                du1x += dlx1[a] * ly1[b] * nu_;
                du1y += lx1[a] * dly1[b] * nu_;
                dv1x += dlx1[a] * ly1[b] * nv_;
                dv1y += lx1[a] * dly1[b] * nv_;
            }
    }
    locate(ox - lam * u1, ox, cx2, xi2, st);
    locate(oy - lam * v1, oy, cy2, eta2, st);
    double lx2[3], dlx2[3], ly2[3], dly2[3];
    lagr(xi2, lx2, dlx2);
    lagr(eta2, ly2, dly2);
    const int ci = i + cx2, cj = j + cy2;
    double Wf[4] = {0, 0, 0, 0}, dWx[4] = {0, 0, 0, 0}, dWy[4] = {0, 0, 0, 0};
    double Df[3] = {0, 0, 0}, dDx[3] = {0, 0, 0}, dDy[3] = {0, 0, 0};
    const int wb2 = O.base(ci, cj);
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double w = lx2[a] * ly2[b], wx = dlx2[a] * ly2[b], wy = lx2[a] * dly2[b];
                const int f = fam_of(a, b), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double v = S.at(win_plane(f) + q, wb2, off);
                    Wf[q] += w * v; dWx[q] += wx * v; dWy[q] += wy * v;
                }
                if constexpr (SCHEME == 0) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const double v = S.at(16 + t * 12 + f * 3 + q, wb2, off);
                        Df[q] += w * v; dDx[q] += wx * v; dDy[q] += wy * v;
                    }
                }
            }
    }
    const int wbP = O.base(i, j);
    if constexpr (SCHEME == 1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) Df[q] = S.at(16 + t * 12 + FAM * 3 + q, wbP, 0);
    }
    // ---- reverse ----
    // compose: rho = rho_f + dp rho_K / (gamma p_K), u = u_f + du, v = v_f + dv, p = p_f + dp,
    // with K the foot (SCHEME 0) or the target (SCHEME 1)
    const double rK = SCHEME == 0 ? Wf[0] : WP.r, pK = SCHEME == 0 ? Wf[3] : WP.p;
    const double qinv = 1.0 / (gamma * pK);
    double lw[4] = {0.0, 0.0, 0.0, 0.0};
    {
        const Prim<double> w{Wf[0] + Df[2] * (rK * qinv), Wf[1] + Df[0], Wf[2] + Df[1], Wf[3] + Df[2]};
        double nu[4];
        if constexpr (FAM != F_EH) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = ws * nuF[k];
            flux_x_T(w, gamma, nu, lw);
        }
        if constexpr (FAM != F_EV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = ws * nuG[k];
            flux_y_T(w, gamma, nu, lw);
        }
        if (extra)
#pragma unroll
            for (int k = 0; k < 4; ++k) lw[k] += extra[k];
    }
    double lWf[4], lDf[3];
    lDf[0] = lw[1];
    lDf[1] = lw[2];
    lDf[2] = lw[3] + lw[0] * rK * qinv;
    lWf[1] = lw[1];
    lWf[2] = lw[2];
    if constexpr (SCHEME == 0) {
        lWf[0] = lw[0] * (1.0 + Df[2] * qinv);
        lWf[3] = lw[3] - lw[0] * Df[2] * rK * qinv / pK;
    } else {
        lWf[0] = lw[0];
        lWf[3] = lw[3];
        // the frozen rho_K / (gamma p_K) at the target, and its own increments
        gself[0] += lw[0] * Df[2] * qinv;
        gself[3] -= lw[0] * Df[2] * rK * qinv / pK;
#pragma unroll
        for (int q = 0; q < 3; ++q) O.addb(16 + t * 12 + FAM * 3 + q, wbP, 0, lDf[q]);
    }
    // Q2 values at the foot -> nodes of the foot cell
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double w = lx2[a] * ly2[b];
                const int f = fam_of(a, b), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) O.addb(win_plane(f) + q, wb2, off, w * lWf[q]);
                if constexpr (SCHEME == 0)
#pragma unroll
                    for (int q = 0; q < 3; ++q) O.addb(16 + t * 12 + f * 3 + q, wb2, off, w * lDf[q]);
            }
    }
    // foot position: xi2 = 2 (off - floor(off)) - 1, off = ox - lam u1
    double lxi2 = 0.0, leta2 = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) { lxi2 += lWf[q] * dWx[q]; leta2 += lWf[q] * dWy[q]; }
    if constexpr (SCHEME == 0)
#pragma unroll
        for (int q = 0; q < 3; ++q) { lxi2 += lDf[q] * dDx[q]; leta2 += lDf[q] * dDy[q]; }
    const double lu1 = -2.0 * lam * lxi2, lv1 = -2.0 * lam * leta2;
    // first stage: u1 = Q2(u) at (xi1, eta1)
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const double w = lx1[a] * ly1[b];
                const int f = fam_of(a, b), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
                O.addb(win_plane(f) + 1, wb1, off, w * lu1);
                O.addb(win_plane(f) + 2, wb1, off, w * lv1);
            }
    }
    const double lxi1 = lu1 * du1x + lv1 * dv1x, leta1 = lu1 * du1y + lv1 * dv1y;
    gself[1] += -2.0 * lam * lxi1;
    gself[2] += -2.0 * lam * leta1;
}

// Forward intermediates of a TX x TY tile, recomputed from state_n for the reverse
// sweep: the tile's primitive node values (node-cells [-1, T+1)) and recovered centres
// (cells [-1, T)) staged in LDS, then the increments of both durations at the tile's
// own node-cells (every wedge of a node-cell in [0, T) lies in cells [-1, T)).  Writes
// W^C of the tile's cells and the 24 increment planes, zeroes the tile's cells of the
// planes the reverse sweep accumulates into, and starts the averages' cotangent at
// cot_np1's (the averages enter the new averages with unit weight).
template <int TX, int TY>
struct IntTile {
    static constexpr int PX = TX + 2, PY = TY + 2, CX = TX + 1, CY = TY + 1;
    double P[12][PY][PX];
    double C[4][CY][CX];
};

template <int TX, int TY>
struct IntAcc {
    const IntTile<TX, TY>* t;
    __device__ __forceinline__ Prim<double> node(int fam, int x, int y) const {
        if (fam == F_C) return {t->C[0][y + 1][x + 1], t->C[1][y + 1][x + 1], t->C[2][y + 1][x + 1], t->C[3][y + 1][x + 1]};
        const int b = 4 * fam;
        return {t->P[b][y + 1][x + 1], t->P[b + 1][y + 1][x + 1], t->P[b + 2][y + 1][x + 1], t->P[b + 3][y + 1][x + 1]};
    }
};

constexpr int kFBX = 32, kFBY = 8, kFNT = kFBX * kFBY;
using FwdTile = IntTile<kFBX, kFBY>;

// two workgroups per CU (256 registers per lane)
struct AvgPlanes { const double* src[4]; double* dst[4]; };

__global__ void __launch_bounds__(kFNT, 2) k_adj_fwd(StatePtrs<double> prim, double* C, double* D, PlaneList Z,
                                                     int nzero, AvgPlanes avg, int nx, int ny, double gamma,
                                                     double lam0, double lam1, unsigned* status) {
    __shared__ FwdTile L;
    const int i0 = blockIdx.x * kFBX, j0 = blockIdx.y * kFBY, tid = threadIdx.x;
    const size_t N = (size_t)nx * ny;
    const int ox = tid % kFBX, oy = tid / kFBX;
    const bool own = i0 + ox < nx && j0 + oy < ny;
    const size_t g = own ? (size_t)(j0 + oy) * nx + (i0 + ox) : 0;
    unsigned st = 0;
    // stage primitives: all loads of a thread's rounds are issued before its stores
    {
        constexpr int NP = FwdTile::PX * FwdTile::PY, R = (NP + kFNT - 1) / kFNT;
        double v[R][12];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = r * kFNT + tid;
            if (e < NP) {
                const size_t k = (size_t)wrap_any(j0 - 1 + e / FwdTile::PX, ny) * nx + wrap_any(i0 - 1 + e % FwdTile::PX, nx);
#pragma unroll
                for (int q = 0; q < 12; ++q) v[r][q] = prim.p[4 + q][k];
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = r * kFNT + tid;
            if (e < NP)
#pragma unroll
                for (int q = 0; q < 12; ++q) L.P[q][e / FwdTile::PX][e % FwdTile::PX] = v[r][q];
        }
    }
    if (own) {
        for (int q = 0; q < nzero; ++q) Z.p[q][g] = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) avg.dst[q][g] = avg.src[q][g];
    }
    __syncthreads();
    // recovered centres of cells [-1, T)
    {
        const IntAcc<kFBX, kFBY> A{&L};
        for (int e = tid; e < FwdTile::CX * FwdTile::CY; e += kFNT) {
            const int x = e % FwdTile::CX - 1, y = e / FwdTile::CX - 1;
            const size_t k = (size_t)wrap_any(j0 + y, ny) * nx + wrap_any(i0 + x, nx);
            const double Ub[4] = {prim.p[0][k], prim.p[1][k], prim.p[2][k], prim.p[3][k]};
            const Prim<double> w = recover_centre(Ub, A.node(F_V, x, y), A.node(F_V, x + 1, y), A.node(F_V, x, y + 1),
                                                  A.node(F_V, x + 1, y + 1), A.node(F_EH, x, y), A.node(F_EH, x, y + 1),
                                                  A.node(F_EV, x, y), A.node(F_EV, x + 1, y), gamma);
            L.C[0][y + 1][x + 1] = w.r;
            L.C[1][y + 1][x + 1] = w.u;
            L.C[2][y + 1][x + 1] = w.v;
            L.C[3][y + 1][x + 1] = w.p;
            if (x >= 0 && y >= 0 && i0 + x < nx && j0 + y < ny) {
                const size_t c = (size_t)(j0 + y) * nx + (i0 + x);
                C[c] = w.r;
                C[N + c] = w.u;
                C[2 * N + c] = w.v;
                C[3 * N + c] = w.p;
                if (!(w.r > 0.0) || !(w.p > 0.0)) st |= SB_NONPHYS;
            }
        }
    }
    __syncthreads();
    // increments of the tile's own node-cells
    if (own) {
        const IntAcc<kFBX, kFBY> A{&L};
        const PolAbs<double> pol{gamma, 1.0 / (gamma - 1.0)};
        double d[2][3];
        node_increments<F_V>(A, ox, oy, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) D[(size_t)(t * 12 + 0 * 3 + v) * N + g] = d[t][v];
        __builtin_amdgcn_sched_barrier(0);   // one family at a time: interleaving them spills
        node_increments<F_EV>(A, ox, oy, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) D[(size_t)(t * 12 + 1 * 3 + v) * N + g] = d[t][v];
        __builtin_amdgcn_sched_barrier(0);
        node_increments<F_EH>(A, ox, oy, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) D[(size_t)(t * 12 + 2 * 3 + v) * N + g] = d[t][v];
        __builtin_amdgcn_sched_barrier(0);
        node_increments<F_C>(A, ox, oy, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) D[(size_t)(t * 12 + 3 * 3 + v) * N + g] = d[t][v];
    }
    if (st) atomicOr(status, st);
}

// Reverse sweep of one target (family FAM of node-cell (i, j)): the adjoints of the
// edge fluxes it feeds, from the averages' cotangents, then of its three time levels
// (w^n directly, w^{n+1/2} and w^{n+1} through the transposed point update).
template <int FAM, int SCHEME, class S_, class O_>
__device__ void point_adj_target(const S_& S, const StatePtrs<double>& cot1, const O_& O, int nx, int ny, int i,
                                 int j, double gamma, double lam0, double lam1) {
    const int im = wrap1(i - 1, nx), jm = wrap1(j - 1, ny);
    auto lU = [&](int a, int b, int k) -> double {
        return cot1.p[k][(size_t)(b == j ? j : jm) * nx + (a == i ? i : im)];
    };
    // cotangents of the time-integrated edge fluxes at this node: F at V and Ev, G at
    // V and Eh; spatial Simpson weights 1/6 (V, two edges each) and 4/6 (edge midpoints)
    double nuF[4] = {0, 0, 0, 0}, nuG[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double muF_ij = lam1 * (lU(i, j, k) - lU(i - 1, j, k));
        const double muG_ij = lam1 * (lU(i, j, k) - lU(i, j - 1, k));
        if constexpr (FAM == F_V) {
            const double muF_ijm = lam1 * (lU(i, j - 1, k) - lU(i - 1, j - 1, k));
            const double muG_imj = lam1 * (lU(i - 1, j, k) - lU(i - 1, j - 1, k));
            nuF[k] = (muF_ij + muF_ijm) * (1.0 / 6.0);
            nuG[k] = (muG_ij + muG_imj) * (1.0 / 6.0);
        } else if constexpr (FAM == F_EV) {
            nuF[k] = muF_ij * (4.0 / 6.0);
        } else {
            nuG[k] = muG_ij * (4.0 / 6.0);
        }
    }
    // time level n (time-Simpson weight 1/6): the node itself
    const int wb = O.base(i, j);
    const Prim<double> w0 = S.node(FAM, wb);
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    {
        double nu[4];
        if constexpr (FAM != F_EH) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = nuF[k] * (1.0 / 6.0);
            flux_x_T(w0, gamma, nu, g);
        }
        if constexpr (FAM != F_EV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = nuG[k] * (1.0 / 6.0);
            flux_y_T(w0, gamma, nu, g);
        }
    }
    // n + 1/2 (weight 4/6) and n + 1 (weight 1/6; also an output of the step)
    point_update_adj<FAM, SCHEME>(S, O, 0, i, j, w0, gamma, lam0, nuF, nuG, 4.0 / 6.0, nullptr, g);
    const size_t c = (size_t)j * nx + i;
    const double extra[4] = {cot1.p[4 + 4 * FAM][c], cot1.p[5 + 4 * FAM][c], cot1.p[6 + 4 * FAM][c],
                             cot1.p[7 + 4 * FAM][c]};
    point_update_adj<FAM, SCHEME>(S, O, 1, i, j, w0, gamma, lam1, nuF, nuG, 1.0 / 6.0, extra, g);
#pragma unroll
    for (int q = 0; q < 4; ++q) O.addb(win_plane(FAM) + q, wb, 0, g[q]);
}

// Reverse of the point update, fluxes and average update for a BX x BY block of
// cells, one thread per (cell, target family).  Feet stay within one cell (guarded),
// so every read of the forward state and every contribution lies in node-cells
// [-1, B + 2) of the block: the block stages the forward state of that window in LDS
// (each thread loads all 40 planes of one node-cell at once) and accumulates into an
// LDS window of the same shape.
// 8x8 blocks: the staged state and the window take 77 KB, so two blocks share a CU and
// one's staging overlaps the other's work (2% faster than 16x8 at one block per CU,
// despite the larger window overlap, 1.89x against 1.63x).
constexpr int kPBX = 8, kPBY = 8, kPNT = 3 * kPBX * kPBY;
constexpr int kPRX = kPBX + 3, kPRY = kPBY + 3, kPWin = kPRX * kPRY;
using PointWin = LdsWin<40, kPRX, kPRY>;
using PointStage = StageWin<kPRX, kPRY>;
constexpr size_t kPointLds = sizeof(double) * 2 * 40 * kPWin;   // staged state + accumulators
static_assert(kPWin <= kPNT, "one staging round");

// (registers bounded for 2 waves per SIMD: the workgroup alone would let the compiler
// take accumulation registers too, and the RB instantiation did, at one wave per SIMD)
template <int SCHEME>
__global__ void __launch_bounds__(kPNT, 2) k_adj_points(StatePtrs<double> prim, const double* C, const double* Dfwd,
                                                     StatePtrs<double> cot1, PlaneList G, int nx, int ny,
                                                     double gamma, double lam0, double lam1) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* stage = reinterpret_cast<double*>(smem);   // [40][RY][RX]
    const int i0 = blockIdx.x * kPBX, j0 = blockIdx.y * kPBY;
    const PointWin O{stage + 40 * kPWin, i0 - 1, j0 - 1};
    O.zero();
    if (threadIdx.x < kPWin) {
        const int e = threadIdx.x;
        const int i = wrap_any(i0 - 1 + e % kPRX, nx), j = wrap_any(j0 - 1 + e / kPRX, ny);
        const size_t N = (size_t)nx * ny, k = (size_t)j * nx + i;
        double v[40];
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) v[pl] = prim.p[4 + pl][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[12 + q] = C[q * N + k];
#pragma unroll
        for (int q = 0; q < 24; ++q) v[16 + q] = Dfwd[q * N + k];
#pragma unroll
        for (int pl = 0; pl < 40; ++pl) stage[pl * kPWin + e] = v[pl];
    }
    __syncthreads();
    const PointStage S{stage, i0 - 1, j0 - 1};
    const int cell = (int)threadIdx.x % (kPBX * kPBY), fam = (int)threadIdx.x / (kPBX * kPBY);   // wave-uniform
    const int i = i0 + cell % kPBX, j = j0 + cell / kPBX;
    if (i < nx && j < ny) {
        if (fam == F_V) point_adj_target<F_V, SCHEME>(S, cot1, O, nx, ny, i, j, gamma, lam0, lam1);
        else if (fam == F_EV) point_adj_target<F_EV, SCHEME>(S, cot1, O, nx, ny, i, j, gamma, lam0, lam1);
        else point_adj_target<F_EH, SCHEME>(S, cot1, O, nx, ny, i, j, gamma, lam0, lam1);
    }
    __syncthreads();
    flush_window(O, G, nx, ny);
}

// Transposed 1-D Lagrange-to-monomial transform (see mono1): (lc0, lc1, lc2) -> (lf0, lf1, lf2).
template <int XC>
__device__ __forceinline__ void mono1_T(double c0, double c1, double c2, double& f0, double& f1, double& f2) {
    if constexpr (XC == 0) { f0 = c0 - 3.0 * c1 + 2.0 * c2; f1 = 4.0 * c1 - 4.0 * c2; f2 = -c1 + 2.0 * c2; }
    else if constexpr (XC == 1) { f0 = c1 + 2.0 * c2; f1 = -4.0 * c1 - 4.0 * c2; f2 = c0 + 3.0 * c1 + 2.0 * c2; }
    else { f0 = -c1 + 2.0 * c2; f1 = c0 - 4.0 * c2; f2 = c1 + 2.0 * c2; }
}

// Transposed wedge: adjoint of the accumulators -> adjoint of the cell's nodal (p, u, v),
// scattered to the nodes of cell (ci, cj).
template <int W, int XC, int YC, class O_>
__device__ __forceinline__ void wedge_adj(const double la[6][4], const O_& O, int ci, int cj) {
    constexpr int RX = O_::kRX;
    double lc[3][3][3];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) lc[v][a][b] = 0.0;
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
            if (al + be == 0) continue;
            const int m = al + be - 1;
            const double* B = kBlk[W][al][be];
            double sp = 0.0, su = 0.0, sv = 0.0;
            if (B[0] != 0.0) sp += B[0] * la[0][m];
            if (B[3] != 0.0) sp += B[3] * la[2][m];
            if (B[6] != 0.0) sp += B[6] * la[4][m];
            if (B[1] != 0.0) su += B[1] * la[1][m];
            if (B[4] != 0.0) su += B[4] * la[3][m];
            if (B[7] != 0.0) su += B[7] * la[5][m];
            if (B[2] != 0.0) sv += B[2] * la[1][m];
            if (B[5] != 0.0) sv += B[5] * la[3][m];
            if (B[8] != 0.0) sv += B[8] * la[5][m];
            lc[0][al][be] = sp;
            lc[1][al][be] = su;
            lc[2][al][be] = sv;
        }
    double lf[3][3][3];   // [var][x-node][y-node]
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        double lg[3][3];  // [alpha][y-node]
#pragma unroll
        for (int al = 0; al < 3; ++al) mono1_T<YC>(lc[v][al][0], lc[v][al][1], lc[v][al][2], lg[al][0], lg[al][1], lg[al][2]);
#pragma unroll
        for (int b = 0; b < 3; ++b) mono1_T<XC>(lg[0][b], lg[1][b], lg[2][b], lf[v][0][b], lf[v][1][b], lf[v][2][b]);
    }
    const int wb = O.base(ci, cj);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int pl = win_plane(fam_of(a, b)), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
            O.addb(pl + 1, wb, off, lf[1][a][b]);
            O.addb(pl + 2, wb, off, lf[2][a][b]);
            O.addb(pl + 3, wb, off, lf[0][a][b]);
        }
}

template <int FAM, class O_>
__device__ void incr_adj(const AdjNodes& A, const O_& O, const double* lD, int i, int j, double gamma, double lam0,
                         double lam1) {
    const size_t N = (size_t)A.nx * A.ny, k = A.idx(i, j);
    double li[2][3];
    bool any = false;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            li[t][q] = lD[(size_t)(t * 12 + FAM * 3 + q) * N + k];
            any = any || (li[t][q] != 0.0);
        }
    if (!any) return;
    const Prim<double> W = A.node(FAM, i, j);
    const double c = sqrt(gamma * W.p / W.r);
    const double Z = W.r * c, iZ = 1.0 / Z;
    NodeAcc<double> na;
    na.zero();
    node_wedges<FAM>(A, i, j, na);
    double la[6][4];
#pragma unroll
    for (int ch = 0; ch < 6; ++ch)
#pragma unroll
        for (int m = 0; m < 4; ++m) la[ch][m] = 0.0;
    double lc = 0.0, lZ = 0.0, liZ = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const double lam = t ? lam1 : lam0;
        const double r = c * lam;
        double s[6], ds[6];
#pragma unroll
        for (int ch = 0; ch < 6; ++ch) {
            s[ch] = ((na.a[ch][3] * r + na.a[ch][2]) * r + na.a[ch][1]) * r + na.a[ch][0];
            ds[ch] = (3.0 * na.a[ch][3] * r + 2.0 * na.a[ch][2]) * r + na.a[ch][1];
        }
        // inc0 = r (s2 iZ + s3), inc1 = r (s4 iZ + s5), inc2 = r (s0 + Z s1)
        double ls[6];
        ls[2] = li[t][0] * r * iZ;
        ls[3] = li[t][0] * r;
        ls[4] = li[t][1] * r * iZ;
        ls[5] = li[t][1] * r;
        ls[0] = li[t][2] * r;
        ls[1] = li[t][2] * r * Z;
        double rp = 1.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int ch = 0; ch < 6; ++ch) la[ch][m] += ls[ch] * rp;
            rp *= r;
        }
        const double lr = li[t][0] * (s[2] * iZ + s[3] + r * (ds[2] * iZ + ds[3])) +
                          li[t][1] * (s[4] * iZ + s[5] + r * (ds[4] * iZ + ds[5])) +
                          li[t][2] * (s[0] + Z * s[1] + r * (ds[0] + Z * ds[1]));
        lc += lam * lr;
        liZ += li[t][0] * r * s[2] + li[t][1] * r * s[4];
        lZ += li[t][2] * r * s[1];
    }
    lZ += -iZ * iZ * liZ;
    // c = sqrt(gamma p / rho), Z = rho c
    {
        const int wb = O.base(i, j);
        O.addb(win_plane(FAM), wb, 0, lc * (-c / (2.0 * W.r)) + lZ * (0.5 * c));
        O.addb(win_plane(FAM) + 3, wb, 0, lc * (c / (2.0 * W.p)) + lZ * (W.r * c / (2.0 * W.p)));
    }
    if constexpr (FAM == F_V) {
        wedge_adj<W_V_NE, 0, 0>(la, O, i, j);
        wedge_adj<W_V_NW, 1, 0>(la, O, i - 1, j);
        wedge_adj<W_V_SW, 1, 1>(la, O, i - 1, j - 1);
        wedge_adj<W_V_SE, 0, 1>(la, O, i, j - 1);
    } else if constexpr (FAM == F_EV) {
        wedge_adj<W_EV_R, 0, 2>(la, O, i, j);
        wedge_adj<W_EV_L, 1, 2>(la, O, i - 1, j);
    } else if constexpr (FAM == F_EH) {
        wedge_adj<W_EH_U, 2, 0>(la, O, i, j);
        wedge_adj<W_EH_D, 2, 1>(la, O, i, j - 1);
    } else {
        wedge_adj<W_C, 2, 2>(la, O, i, j);
    }
}

__device__ __forceinline__ void cons_T(const Prim<double>& w, double gamma, const double lU[4], double g[4]) {
    // U = (rho, rho u, rho v, p/(gamma-1) + rho (u^2+v^2)/2)
    const double q2 = 0.5 * (w.u * w.u + w.v * w.v);
    g[0] = lU[0] + w.u * lU[1] + w.v * lU[2] + q2 * lU[3];
    g[1] = w.r * lU[1] + w.r * w.u * lU[3];
    g[2] = w.r * lU[2] + w.r * w.v * lU[3];
    g[3] = lU[3] / (gamma - 1.0);
}

// Transposed centre recovery of cell (i, j) for the centre cotangent lW: the averages'
// cotangent (plane 16 + k of the window, weight 9/4) and the point values of the cell's
// eight boundary nodes (through U(W) at corners, weight -1/16, and edge midpoints, -1/4).
template <class O_>
__device__ __forceinline__ void centre_adj(const AdjNodes& A, const O_& O, int i, int j, const double lW[4],
                                           double gamma) {
    const Prim<double> Wc = A.node(F_C, i, j);
    // W = prim(U_c): rho = U0, u = U1/U0, v = U2/U0, p = (g-1)(U3 - (U1 u + U2 v)/2)
    const double ir = 1.0 / Wc.r, gm1 = gamma - 1.0;
    double lU[4];
    lU[0] = lW[0] - lW[1] * Wc.u * ir - lW[2] * Wc.v * ir + lW[3] * gm1 * 0.5 * (Wc.u * Wc.u + Wc.v * Wc.v);
    lU[1] = lW[1] * ir - lW[3] * gm1 * Wc.u;
    lU[2] = lW[2] * ir - lW[3] * gm1 * Wc.v;
    lU[3] = lW[3] * gm1;
    // U_c = 9/4 [Ubar - sum_corners U / 36 - sum_edges U / 9]
    const int wb = O.base(i, j);
#pragma unroll
    for (int k = 0; k < 4; ++k) O.addb(16 + k, wb, 0, 2.25 * lU[k]);
    double lc[4], le[4], g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { lc[k] = -lU[k] * (1.0 / 16.0); le[k] = -lU[k] * 0.25; }
    cons_T(A.node(F_V, i, j), gamma, lc, g);          O.node(F_V, i, j, g);
    cons_T(A.node(F_V, i + 1, j), gamma, lc, g);      O.node(F_V, i + 1, j, g);
    cons_T(A.node(F_V, i, j + 1), gamma, lc, g);      O.node(F_V, i, j + 1, g);
    cons_T(A.node(F_V, i + 1, j + 1), gamma, lc, g);  O.node(F_V, i + 1, j + 1, g);
    cons_T(A.node(F_EH, i, j), gamma, le, g);         O.node(F_EH, i, j, g);
    cons_T(A.node(F_EH, i, j + 1), gamma, le, g);     O.node(F_EH, i, j + 1, g);
    cons_T(A.node(F_EV, i, j), gamma, le, g);         O.node(F_EV, i, j, g);
    cons_T(A.node(F_EV, i + 1, j), gamma, le, g);     O.node(F_EV, i + 1, j, g);
}

// Transposed node increments and centre recovery for a BX x BY block of node-cells.
// Every wedge of a node-cell in [0, B) lies in cells [-1, B) and its nodes in node-cells
// [-1, B + 1): an LDS window over those node-cells collects the point-value, centre and
// averages' contributions.  The centre recovery is linear in the centre cotangent, so
// the block applies its transpose to the centre contributions of its own increments
// (window cells [-1, B)) plus, for its own cells, the centre cotangent the point kernel
// left in global memory; the neighbouring blocks do the same with theirs, and the sum
// is the transpose applied to the total.  The centre nodes of those cells and their
// boundary nodes stay inside the window.
constexpr int kIBX = 32, kIBY = 8;
using IncrWin = LdsWin<20, kIBX + 2, kIBY + 2>;   // planes 0..15 as the point window, 16..19 averages

__global__ void __launch_bounds__(kIBX * kIBY, 2) k_adj_incr(StatePtrs<double> prim, const double* C, const double* lD,
                                                          const double* lC, PlaneList G, int nx, int ny,
                                                          double gamma, double lam0, double lam1) {
    __shared__ double win[20 * (kIBX + 2) * (kIBY + 2)];
    const int i0 = blockIdx.x * kIBX, j0 = blockIdx.y * kIBY;
    const IncrWin O{win, i0 - 1, j0 - 1};
    O.zero();
    __syncthreads();
    AdjNodes A{{}, C, nx, ny};
#pragma unroll
    for (int k = 0; k < 16; ++k) A.s[k] = prim.p[k];
    {
        const int i = i0 + (int)threadIdx.x % kIBX;
        const int j = j0 + (int)threadIdx.x / kIBX;
        if (i < nx && j < ny) {
            incr_adj<F_V>(A, O, lD, i, j, gamma, lam0, lam1);
            incr_adj<F_EV>(A, O, lD, i, j, gamma, lam0, lam1);
            incr_adj<F_EH>(A, O, lD, i, j, gamma, lam0, lam1);
            incr_adj<F_C>(A, O, lD, i, j, gamma, lam0, lam1);
        }
    }
    __syncthreads();
    // cells [-1, B): each centre entry is read (and cleared, so that the flush skips it)
    // by one thread, which scatters into other planes only
    const size_t N = (size_t)nx * ny;
    constexpr int CW = kIBX + 1, CH = kIBY + 1;
    for (int e = threadIdx.x; e < CW * CH; e += blockDim.x) {
        const int i = i0 - 1 + e % CW, j = j0 - 1 + e / CW;
        // past a ragged grid edge the window holds no contributions (the block's
        // node-cells there are skipped), and the cell would index outside the grid
        if (i >= nx || j >= ny) continue;
        const bool own = i >= i0 && j >= j0 && i < nx && j < ny;
        const int wb = O.base(i, j);
        double lW[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            double* c = O.a + wb + (12 + k) * IncrWin::kPlane;
            lW[k] = *c + (own ? lC[k * N + (size_t)j * nx + i] : 0.0);
            *c = 0.0;
        }
        centre_adj(A, O, i, j, lW, gamma);
    }
    __syncthreads();
    flush_window(O, G, nx, ny);
}

hipError_t launch_adjoint_f64(const StepArgs& a, const void* const cot1_[16], void* const cot0_[16]) {
    const size_t N = (size_t)a.nx * a.ny;
    double* C = (double*)a.scratch;
    double* Dfwd = C + 4 * N;
    double* lC = Dfwd + 24 * N;
    double* lD = lC + 4 * N;
    StatePtrs<double> prim, cot1, cot0;
    for (int k = 0; k < 16; ++k) {
        prim.p[k] = (double*)a.in[k];
        cot1.p[k] = (double*)cot1_[k];
        cot0.p[k] = (double*)cot0_[k];
    }
    PlaneList L;
    int np = 0;
    for (int k = 4; k < 16; ++k) L.p[np++] = cot0.p[k];
    for (int k = 0; k < 4; ++k) L.p[np++] = lC + k * N;
    for (int k = 0; k < 24; ++k) L.p[np++] = lD + k * N;
    // L lists the window planes in LdsWin order: point values, centres, increments
    PlaneList Li = L;   // k_adj_incr's window: point values, centres (consumed in the block), averages
    for (int k = 0; k < 4; ++k) Li.p[16 + k] = cot0.p[k];
    AvgPlanes avg;
    for (int k = 0; k < 4; ++k) { avg.src[k] = cot1.p[k]; avg.dst[k] = cot0.p[k]; }
    const double lam1 = a.dt / a.h, lam0 = 0.5 * lam1;
    {
        dim3 grd((a.nx + kFBX - 1) / kFBX, (a.ny + kFBY - 1) / kFBY);
        hipLaunchKernelGGL(k_adj_fwd, grd, dim3(kFNT), 0, a.stream, prim, C, Dfwd, L, np, avg, a.nx, a.ny, a.gamma,
                           lam0, lam1, a.status);
    }
    if (a.ev_begin) (void)hipEventRecord(a.ev_begin, a.stream);
    {
        const size_t lds = kPointLds;   // allowed by prepare_adjoint_f64
        dim3 grd((a.nx + kPBX - 1) / kPBX, (a.ny + kPBY - 1) / kPBY);
        if (a.scheme == 0)
            hipLaunchKernelGGL(k_adj_points<0>, grd, dim3(kPNT), lds, a.stream, prim, C, Dfwd, cot1, L, a.nx, a.ny,
                               a.gamma, lam0, lam1);
        else
            hipLaunchKernelGGL(k_adj_points<1>, grd, dim3(kPNT), lds, a.stream, prim, C, Dfwd, cot1, L, a.nx, a.ny,
                               a.gamma, lam0, lam1);
    }
    {
        dim3 grd((a.nx + kIBX - 1) / kIBX, (a.ny + kIBY - 1) / kIBY);
        hipLaunchKernelGGL(k_adj_incr, grd, dim3(kIBX * kIBY), 0, a.stream, prim, C, lD, lC, Li, a.nx, a.ny, a.gamma,
                           lam0, lam1);
    }
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    return hipGetLastError();
}

hipError_t prepare_adjoint_f64() {
    const hipError_t e = hipFuncSetAttribute((const void*)k_adj_points<0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)kPointLds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_adj_points<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kPointLds);
}

size_t scratch_bytes_adjoint_f64(int nx, int ny) { return (size_t)nx * ny * (4 + 24 + 4 + 24) * sizeof(double); }

}  // namespace af
