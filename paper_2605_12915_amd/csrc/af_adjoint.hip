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

#include <mutex>

#include "af_adjoint.h"
#include "af_internal.h"

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

// Cotangent planes read by cell with a periodic wrap of at most one grid length.
struct CotAcc {
    StatePtrs<double> s;
    int nx, ny;
    __device__ __forceinline__ double get(int k, int i, int j) const {
        i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
        j = (j < 0) ? j + ny : (j >= ny ? j - ny : j);
        return s.p[k][(size_t)j * nx + i];
    }
};

// One buffer of consecutive planes read by cell (the increments' cotangent).
struct PlanesAcc {
    const double* base;
    int nx, ny;
    __device__ __forceinline__ double get(int k, int i, int j) const {
        i = (i < 0) ? i + nx : (i >= nx ? i - nx : i);
        j = (j < 0) ? j + ny : (j >= ny ? j - ny : j);
        return base[(size_t)k * nx * ny + (size_t)j * nx + i];
    }
};

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

// Periodic index: one shift (offsets of at most one grid length) or a modulo.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int wrap_any(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
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

// XCD-aware workgroup numbering (as in the step kernels): workgroup b runs on XCD
// b mod 8; each XCD takes a contiguous run of the row-major block list, so that the
// overlapping halos and accumulation windows of neighbouring blocks meet in one L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
    const int xcd = b & 7;
    int base = 0;
    for (int x = 0; x < xcd; ++x) base += (ntiles - x + 7) >> 3;
    return base + (b >> 3);
}

constexpr int kFBX = 32, kFBY = 8, kFNT = kFBX * kFBY;
using FwdTile = IntTile<kFBX, kFBY>;

// two workgroups per CU (256 registers per lane)
struct AvgPlanes { const double* src[4]; double* dst[4]; };

__global__ void __launch_bounds__(kFNT, 2) k_adj_fwd(StatePtrs<double> prim, double* C, double* D, PlaneList Z,
                                                     int nzero, AvgPlanes avg, int nx, int ny, int tiles_x, int ntiles,
                                                     double gamma, double lam0, double lam1, unsigned* status) {
    __shared__ FwdTile L;
    const int tile = xcd_tile(blockIdx.x, ntiles), tid = threadIdx.x;
    const int i0 = (tile % tiles_x) * kFBX, j0 = (tile / tiles_x) * kFBY;
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

// Reverse of the point update, fluxes and average update for a BX x BY block of
// cells, one thread per (cell, target family).  Feet stay within one cell (guarded),
// so every read of the forward state and every contribution lies in node-cells
// [-1, B + 2) of the block: the block stages the forward state of that window in LDS
// (each thread loads all 40 planes of one node-cell at once) and accumulates into an
// LDS window of the same shape.
// 8x8 blocks: the staged state and the window take 79 KB, so two blocks share a CU and
// one's staging overlaps the other's work (2% faster than 16x8 at one block per CU,
// despite the larger window overlap, 1.89x against 1.63x).
// The accumulation window's rows are padded to WX = 12 doubles (its twelfth column is
// never written): with the block's rows split between the half-wavefronts as
// {0, 2, 4, 6} and {1, 3, 5, 7}, the four rows a half-wavefront adds to at a common
// offset start 0, 24, 48 and 72 doubles apart, i.e. in four distinct quarters of the
// 64 LDS banks (with 11-double rows, rows 0 and 3 of four consecutive ones collide).
template <int BX, int BY>
struct PointBlock {
    static constexpr int NT = 3 * BX * BY, RX = BX + 3, RY = BY + 3, WIN = RX * RY;
    static constexpr int WX = BX == 8 ? 12 : RX, WWIN = WX * RY;
    static constexpr size_t LDS = sizeof(double) * 40 * (WIN + WWIN);   // staged state + accumulators
    static_assert(WIN <= NT, "one staging round");
    static_assert((BX * BY) % 64 == 0, "each wavefront holds one target family");
};

// (registers bounded for MINB blocks per CU at 2 waves per SIMD: the workgroup alone
// would let the compiler take accumulation registers too, and the RB instantiation did,
// at one wave per SIMD)
template <int SCHEME, int BX, int BY, int MINB>
__global__ void __launch_bounds__(3 * BX * BY, MINB)
    k_adj_points(StatePtrs<double> prim, const double* C, const double* Dfwd, StatePtrs<double> cot1, PlaneList G,
                 int nx, int ny, int tiles_x, int ntiles, double gamma, double lam0, double lam1) {
    using B = PointBlock<BX, BY>;
    extern __shared__ __align__(16) unsigned char smem[];
    double* stage = reinterpret_cast<double*>(smem);   // [40][RY][RX]
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int i0 = (tile % tiles_x) * BX, j0 = (tile / tiles_x) * BY;
    const LdsWin<40, B::WX, B::RY> O{stage + 40 * B::WIN, i0 - 1, j0 - 1};
    O.zero();
    if (threadIdx.x < B::WIN) {
        const int e = threadIdx.x;
        const int i = wrap_any(i0 - 1 + e % B::RX, nx), j = wrap_any(j0 - 1 + e / B::RX, ny);
        const size_t N = (size_t)nx * ny, k = (size_t)j * nx + i;
        double v[40];
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) v[pl] = prim.p[4 + pl][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[12 + q] = C[q * N + k];
#pragma unroll
        for (int q = 0; q < 24; ++q) v[16 + q] = Dfwd[q * N + k];
#pragma unroll
        for (int pl = 0; pl < 40; ++pl) stage[pl * B::WIN + e] = v[pl];
    }
    __syncthreads();
    const StageWin<B::RX, B::RY> S{stage, i0 - 1, j0 - 1};
    const int cell = (int)threadIdx.x % (BX * BY), fam = (int)threadIdx.x / (BX * BY);   // wave-uniform
    // rows of a half-wavefront: even rows in the first, odd rows in the second (8x8)
    const int row = BX == 8 && BY == 8 ? 2 * ((cell / 8) % 4) + cell / 32 : cell / BX;
    const int i = i0 + cell % BX, j = j0 + row;
    if (i < nx && j < ny) {
        const CotAcc C1{cot1, nx, ny};
        unsigned fix;
        if (fam == F_V) fix = point_adj_target<F_V, SCHEME, 0>(S, C1, O, i, j, gamma, lam0, lam1);
        else if (fam == F_EV) fix = point_adj_target<F_EV, SCHEME, 0>(S, C1, O, i, j, gamma, lam0, lam1);
        else fix = point_adj_target<F_EH, SCHEME, 0>(S, C1, O, i, j, gamma, lam0, lam1);
        // targets whose Picard stages left one cell (rare): their first-stage share
        if (__any(fix != 0u)) {
            if (fam == F_V) point_adj_target<F_V, SCHEME, 1>(S, C1, O, i, j, gamma, lam0, lam1, fix);
            else if (fam == F_EV) point_adj_target<F_EV, SCHEME, 1>(S, C1, O, i, j, gamma, lam0, lam1, fix);
            else point_adj_target<F_EH, SCHEME, 1>(S, C1, O, i, j, gamma, lam0, lam1, fix);
        }
    }
    __syncthreads();
    flush_window(O, G, nx, ny);
}

template <int SCHEME, int BX, int BY, int MINB>
void launch_points(const StepArgs& a, StatePtrs<double> prim, const double* C, const double* Dfwd,
                   StatePtrs<double> cot1, const PlaneList& L, double lam0, double lam1) {
    using B = PointBlock<BX, BY>;
    const int tx = (a.nx + BX - 1) / BX, nt = tx * ((a.ny + BY - 1) / BY);
    hipLaunchKernelGGL((k_adj_points<SCHEME, BX, BY, MINB>), dim3(nt), dim3(B::NT), B::LDS, a.stream, prim, C, Dfwd,
                       cot1, L, a.nx, a.ny, tx, nt, a.gamma, lam0, lam1);
}

template <int BX, int BY, int MINB>
hipError_t prepare_points() {
    using B = PointBlock<BX, BY>;
    hipError_t e = hipFuncSetAttribute((const void*)k_adj_points<0, BX, BY, MINB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)B::LDS);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_adj_points<1, BX, BY, MINB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)B::LDS);
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
                                                          int tiles_x, int ntiles, double gamma, double lam0,
                                                          double lam1) {
    __shared__ double win[20 * (kIBX + 2) * (kIBY + 2)];
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int i0 = (tile % tiles_x) * kIBX, j0 = (tile / tiles_x) * kIBY;
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
            const PlanesAcc LD{lD, nx, ny};
            incr_adj<F_V>(A, LD, O, i, j, gamma, lam0, lam1);
            incr_adj<F_EV>(A, LD, O, i, j, gamma, lam0, lam1);
            incr_adj<F_EH>(A, LD, O, i, j, gamma, lam0, lam1);
            incr_adj<F_C>(A, LD, O, i, j, gamma, lam0, lam1);
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
        const int tx = (a.nx + kFBX - 1) / kFBX, nt = tx * ((a.ny + kFBY - 1) / kFBY);
        hipLaunchKernelGGL(k_adj_fwd, dim3(nt), dim3(kFNT), 0, a.stream, prim, C, Dfwd, L, np, avg, a.nx, a.ny, tx, nt,
                           a.gamma, lam0, lam1, a.status);
    }
    if (a.ev_begin) (void)hipEventRecord(a.ev_begin, a.stream);
    // point kernel: 8x8-cell blocks, two per CU (16x8 blocks at one per CU, whose
    // half-wavefronts read rows of 16 consecutive words, measured 3% slower)
    if (a.scheme == 0) launch_points<0, 8, 8, 2>(a, prim, C, Dfwd, cot1, L, lam0, lam1);
    else launch_points<1, 8, 8, 2>(a, prim, C, Dfwd, cot1, L, lam0, lam1);
    {
        const int tx = (a.nx + kIBX - 1) / kIBX, nt = tx * ((a.ny + kIBY - 1) / kIBY);
        hipLaunchKernelGGL(k_adj_incr, dim3(nt), dim3(kIBX * kIBY), 0, a.stream, prim, C, lD, lC, Li, a.nx, a.ny, tx, nt,
                           a.gamma, lam0, lam1);
    }
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    return hipGetLastError();
}

hipError_t prepare_adjoint_f64() { return prepare_points<8, 8, 2>(); }

size_t scratch_bytes_adjoint_f64(int nx, int ny) { return (size_t)nx * ny * (4 + 24 + 4 + 24) * sizeof(double); }

// ---- allocation-free form of the adjoint step ------------------------------------
// The scratch of launch_adjoint_f64 (56 planes: forward intermediates and reverse
// accumulators) and the status word, in a file-scope device array sized for grids of
// up to kNoallocMaxCells cells.  Every device that loads the library holds its own copy
// for the life of the process.  Only its device address (hipGetSymbolAddress, taken
// once per device with that device current) is ever handed to kernels; the array's name
// in host code is a host-side stand-in.  k_adj_fwd zeroes every accumulation plane for
// the grid's cells itself; the status word is cleared by a fill kernel on each call.
constexpr size_t kNoallocStatusWords = 32;   // 256 bytes: the planes stay 256-byte aligned
static __device__ __align__(256) double scratch[kNoallocStatusWords + kNoallocMaxCells * 56];

static_assert(sizeof(scratch) == kNoallocBytes, "scratch size as declared in af_internal.h");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
void* g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        // the point kernel's LDS exceeds the default limit: allowed once per device here
        e = prepare_adjoint_f64();
        if (e != hipSuccess) return e;
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return hipSuccess;
}

hipError_t launch_adjoint_noalloc(StepArgs a, const void* const cot1[16], void* const cot0[16]) {
    void* p = nullptr;
    hipError_t e = noalloc_scratch_ptr(&p);
    if (e != hipSuccess) return e;
    a.status = (unsigned*)p;
    a.scratch = (double*)p + kNoallocStatusWords;
    e = launch_zero(p, kNoallocStatusWords * sizeof(double), a.stream);
    if (e != hipSuccess) return e;
    return launch_adjoint_f64(a, cot1, cot0);
}

}  // namespace af
