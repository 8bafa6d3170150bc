// Two-launch RB-TAI step, FP64, gfx950: the acoustic increments are computed once
// per node (no halo recompute) and handed to the point/flux kernel through HBM.
//
//   k_acoustic   tile of cells: stage the primitive nodes of node-cells [-1, T+1)^2
//                in LDS, recover the centres of cells [-1, T)^2 (eq. center-node),
//                then the increments of V, Ev, Eh, C of the owned node-cells for
//                tau = dt/2 and dt (App. D).  Writes W^C (4 planes) and the
//                increments (24 planes).
//   k_points     tile of cells: stage the primitive nodes, centres and increments of
//                node-cells [-1, T+2)^2, transported point updates of the targets of
//                node-cells [0, T] (Sec. 6.1 steps 3-4), time-Simpson fluxes per
//                target, then the spatial Simpson fluxes and the average update of
//                the owned cells (eq. af-average-update), all from the same tile.
#include <hip/hip_runtime.h>

#include "af_internal.h"
#include "af_kernels.h"

namespace af {

__device__ __forceinline__ int wrap_n(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// LDS view: node-cell (x, y) of family fam at P[4 fam + k][y + O][x + O],
// centre at C[k][y + OC][x + OC].
template <int PX, int PY, int O, int CXD, int CYD, int OC>
struct PCView {
    const double (*P)[PY][PX];
    const double (*C)[CYD][CXD];
    __device__ __forceinline__ Prim<double> node(int fam, int x, int y) const {
        if (fam == F_C) return {C[0][y + OC][x + OC], C[1][y + OC][x + OC], C[2][y + OC][x + OC], C[3][y + OC][x + OC]};
        const int b = 4 * fam;
        return {P[b][y + O][x + O], P[b + 1][y + O][x + O], P[b + 2][y + O][x + O], P[b + 3][y + O][x + O]};
    }
};

template <int DXD, int DYD, int O>
struct DView {
    const double (*D)[DYD][DXD];    // 12 planes [fam*3 + var] for one tau
    __device__ __forceinline__ double inc(int fam, int x, int y, int var) const { return D[fam * 3 + var][y + O][x + O]; }
};

__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
    const int xcd = b & 7;
    int base = 0;
    for (int x = 0; x < xcd; ++x) base += (ntiles - x + 7) >> 3;
    return base + (b >> 3);
}

// ---------------------------------------------------------------------------------
template <int TX, int TY>
struct AcTile {
    static constexpr int PX = TX + 2, PY = TY + 2;   // node-cells [-1, T+1)
    static constexpr int CX = TX + 1, CY = TY + 1;   // cells [-1, T)
    double P[12][PY][PX];
    double C[4][CY][CX];
};

template <int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_acoustic(StatePtrs<double> in, double* Cout, double* Dout, int nx, int ny,
                                                 int tiles_x, int ntiles, double gamma, double lam0, double lam1,
                                                 unsigned* status) {
    const PolAbs<double> pol{gamma, 1.0 / (gamma - 1.0)};
    using Tile = AcTile<TX, TY>;
    __shared__ Tile T;
    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int i0 = (tile % tiles_x) * TX, j0 = (tile / tiles_x) * TY;
    unsigned st = 0;
    for (int e = tid; e < Tile::PX * Tile::PY; e += NT) {
        const int x = e % Tile::PX, y = e / Tile::PX;
        const size_t g = (size_t)wrap_n(j0 + y - 1, ny) * nx + wrap_n(i0 + x - 1, nx);
#pragma unroll
        for (int k = 0; k < 12; ++k) T.P[k][y][x] = in.p[4 + k][g];
    }
    __syncthreads();
    using View = PCView<Tile::PX, Tile::PY, 1, Tile::CX, Tile::CY, 1>;
    View A{T.P, T.C};
    const size_t N = (size_t)nx * ny;
    for (int e = tid; e < Tile::CX * Tile::CY; e += NT) {
        const int x = e % Tile::CX - 1, y = e / Tile::CX - 1;
        const size_t g = (size_t)wrap_n(j0 + y, ny) * nx + wrap_n(i0 + x, nx);
        const double Ub[4] = {in.p[0][g], in.p[1][g], in.p[2][g], in.p[3][g]};
        Prim<double> w = recover_centre(Ub, A.node(F_V, x, y), A.node(F_V, x + 1, y), A.node(F_V, x, y + 1),
                                        A.node(F_V, x + 1, y + 1), A.node(F_EH, x, y), A.node(F_EH, x, y + 1),
                                        A.node(F_EV, x, y), A.node(F_EV, x + 1, y), gamma);
        T.C[0][y + 1][x + 1] = w.r;
        T.C[1][y + 1][x + 1] = w.u;
        T.C[2][y + 1][x + 1] = w.v;
        T.C[3][y + 1][x + 1] = w.p;
        if (x >= 0 && y >= 0 && i0 + x < nx && j0 + y < ny) {
            if (!(w.r > 0.0) || !(w.p > 0.0)) st |= SB_NONPHYS;
            Cout[g] = w.r;
            Cout[N + g] = w.u;
            Cout[2 * N + g] = w.v;
            Cout[3 * N + g] = w.p;
        }
    }
    __syncthreads();
    for (int e = tid; e < TX * TY; e += NT) {
        const int x = e % TX, y = e / TX;
        if (i0 + x >= nx || j0 + y >= ny) continue;
        const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
        double d[2][3];
        node_increments<F_V>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) Dout[(size_t)(t * 12 + 0 + v) * N + g] = d[t][v];
        node_increments<F_EV>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) Dout[(size_t)(t * 12 + 3 + v) * N + g] = d[t][v];
        node_increments<F_EH>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) Dout[(size_t)(t * 12 + 6 + v) * N + g] = d[t][v];
        node_increments<F_C>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int v = 0; v < 3; ++v) Dout[(size_t)(t * 12 + 9 + v) * N + g] = d[t][v];
    }
    if (st) atomicOr(status, st);
}

// ---------------------------------------------------------------------------------
template <int TX, int TY>
struct PtTile {
    static constexpr int PX = TX + 3, PY = TY + 3;   // node-cells [-1, T+2)
    static constexpr int CX = TX + 2, CY = TY + 2;   // cells [-1, T+1)
    static constexpr int VX = TX + 1, VY = TY + 1;   // flux nodes [0, T]
    double P[12][PY][PX];
    double C[4][CY][CX];
    union {
        double D[2][12][PY][PX];
        struct {
            double FV[8][VY][VX];
            double FE[4][TY][VX];
            double GE[4][VY][TX];
        } F;
    };
};

template <int TX, int TY, int NT, int SCHEME>
__global__ void __launch_bounds__(NT) k_points_update(StatePtrs<double> in, const double* Cin, const double* Din,
                                                      StatePtrs<double> out, int nx, int ny, int tiles_x, int ntiles,
                                                      double gamma, double lam0, double lam1, unsigned* status) {
    const PolAbs<double> pol{gamma, 1.0 / (gamma - 1.0)};
    using Tile = PtTile<TX, TY>;
    extern __shared__ __align__(16) unsigned char smem[];
    Tile& T = *reinterpret_cast<Tile*>(smem);
    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, ntiles);
    const int i0 = (tile % tiles_x) * TX, j0 = (tile / tiles_x) * TY;
    const size_t N = (size_t)nx * ny;
    unsigned st = 0;
    for (int e = tid; e < Tile::PX * Tile::PY; e += NT) {
        const int x = e % Tile::PX, y = e / Tile::PX;
        const size_t g = (size_t)wrap_n(j0 + y - 1, ny) * nx + wrap_n(i0 + x - 1, nx);
#pragma unroll
        for (int k = 0; k < 12; ++k) T.P[k][y][x] = in.p[4 + k][g];
#pragma unroll
        for (int k = 0; k < 24; ++k) (&T.D[0][0][0][0])[(size_t)k * Tile::PY * Tile::PX + y * Tile::PX + x] = Din[k * N + g];
        if (x < Tile::CX && y < Tile::CY) {
#pragma unroll
            for (int k = 0; k < 4; ++k) T.C[k][y][x] = Cin[k * N + g];
        }
    }
    __syncthreads();
    using View = PCView<Tile::PX, Tile::PY, 1, Tile::CX, Tile::CY, 1>;
    View A{T.P, T.C};
    DView<Tile::PX, Tile::PY, 1> D0{T.D[0]}, D1{T.D[1]};
    constexpr int NV_ = Tile::VX * Tile::VY, NE_ = Tile::VX * TY, NH_ = TX * Tile::VY;
    constexpr int NITEMS = NV_ + NE_ + NH_;
    constexpr int ROUNDS = (NITEMS + NT - 1) / NT;
    double fres[ROUNDS][8];
    const double gm1inv = 1.0 / (gamma - 1.0);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int e = r * NT + tid;
        if (e >= NITEMS) continue;
        int fam, x, y;
        if (e < NV_) { fam = F_V; x = e % Tile::VX; y = e / Tile::VX; }
        else if (e < NV_ + NE_) { fam = F_EV; x = (e - NV_) % Tile::VX; y = (e - NV_) / Tile::VX; }
        else { fam = F_EH; x = (e - NV_ - NE_) % TX; y = (e - NV_ - NE_) / TX; }
        Prim<double> w0, wh, w1;
        if (fam == F_V) {
            w0 = A.node(F_V, x, y);
            wh = point_update<F_V, SCHEME>(A, D0, x, y, pol, lam0, st);
            w1 = point_update<F_V, SCHEME>(A, D1, x, y, pol, lam1, st);
        } else if (fam == F_EV) {
            w0 = A.node(F_EV, x, y);
            wh = point_update<F_EV, SCHEME>(A, D0, x, y, pol, lam0, st);
            w1 = point_update<F_EV, SCHEME>(A, D1, x, y, pol, lam1, st);
        } else {
            w0 = A.node(F_EH, x, y);
            wh = point_update<F_EH, SCHEME>(A, D0, x, y, pol, lam0, st);
            w1 = point_update<F_EH, SCHEME>(A, D1, x, y, pol, lam1, st);
        }
        if (x < TX && y < TY && i0 + x < nx && j0 + y < ny) {
            const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
            const int b = 4 + 4 * fam;
            out.p[b][g] = w1.r;
            out.p[b + 1][g] = w1.u;
            out.p[b + 2][g] = w1.v;
            out.p[b + 3][g] = w1.p;
        }
        double F0[4], Fh[4], F1[4];
        if (fam != F_EH) {
            flux_x(w0, gm1inv, F0); flux_x(wh, gm1inv, Fh); flux_x(w1, gm1inv, F1);
#pragma unroll
            for (int k = 0; k < 4; ++k) fres[r][k] = (F0[k] + 4.0 * Fh[k] + F1[k]) * (1.0 / 6.0);
        }
        if (fam != F_EV) {
            flux_y(w0, gm1inv, F0); flux_y(wh, gm1inv, Fh); flux_y(w1, gm1inv, F1);
            const int o = (fam == F_V) ? 4 : 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) fres[r][o + k] = (F0[k] + 4.0 * Fh[k] + F1[k]) * (1.0 / 6.0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int e = r * NT + tid;
        if (e >= NITEMS) continue;
        if (e < NV_) {
            const int x = e % Tile::VX, y = e / Tile::VX;
#pragma unroll
            for (int k = 0; k < 8; ++k) T.F.FV[k][y][x] = fres[r][k];
        } else if (e < NV_ + NE_) {
            const int x = (e - NV_) % Tile::VX, y = (e - NV_) / Tile::VX;
#pragma unroll
            for (int k = 0; k < 4; ++k) T.F.FE[k][y][x] = fres[r][k];
        } else {
            const int x = (e - NV_ - NE_) % TX, y = (e - NV_ - NE_) / TX;
#pragma unroll
            for (int k = 0; k < 4; ++k) T.F.GE[k][y][x] = fres[r][k];
        }
    }
    __syncthreads();
    for (int e = tid; e < TX * TY; e += NT) {
        const int x = e % TX, y = e / TX;
        if (i0 + x >= nx || j0 + y >= ny) continue;
        const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double Fl = (T.F.FV[k][y][x] + 4.0 * T.F.FE[k][y][x] + T.F.FV[k][y + 1][x]) * (1.0 / 6.0);
            const double Fr = (T.F.FV[k][y][x + 1] + 4.0 * T.F.FE[k][y][x + 1] + T.F.FV[k][y + 1][x + 1]) * (1.0 / 6.0);
            const double Gb = (T.F.FV[4 + k][y][x] + 4.0 * T.F.GE[k][y][x] + T.F.FV[4 + k][y][x + 1]) * (1.0 / 6.0);
            const double Gt = (T.F.FV[4 + k][y + 1][x] + 4.0 * T.F.GE[k][y + 1][x] + T.F.FV[4 + k][y + 1][x + 1]) * (1.0 / 6.0);
            out.p[k][g] = in.p[k][g] - lam1 * ((Fr - Fl) + (Gt - Gb));
        }
    }
    if (st) atomicOr(status, st);
}

constexpr int kATX = 32, kATY = 8, kANT = 256;     // acoustic kernel tile
constexpr int kPTX = 32, kPTY = 8, kPNT = 512;     // point/update kernel tile

hipError_t launch_step_split_f64(const StepArgs& a) {
    StatePtrs<double> in, out;
    for (int k = 0; k < 16; ++k) { in.p[k] = (double*)a.in[k]; out.p[k] = (double*)a.out[k]; }
    const size_t N = (size_t)a.nx * a.ny;
    double* C = (double*)a.scratch;
    double* D = C + 4 * N;
    const double lam1 = a.dt / a.h, lam0 = 0.5 * lam1;
    {
        const int tx = (a.nx + kATX - 1) / kATX, ty = (a.ny + kATY - 1) / kATY;
        hipLaunchKernelGGL((k_acoustic<kATX, kATY, kANT>), dim3(tx * ty), dim3(kANT), 0, a.stream, in, C, D, a.nx,
                           a.ny, tx, tx * ty, a.gamma, lam0, lam1, a.status);
    }
    const int tx = (a.nx + kPTX - 1) / kPTX, ty = (a.ny + kPTY - 1) / kPTY;
    const size_t lds = sizeof(PtTile<kPTX, kPTY>);
    if (a.ev_begin) (void)hipEventRecord(a.ev_begin, a.stream);
    if (a.scheme == 0)
        hipLaunchKernelGGL((k_points_update<kPTX, kPTY, kPNT, 0>), dim3(tx * ty), dim3(kPNT), lds, a.stream, in, C, D,
                           out, a.nx, a.ny, tx, tx * ty, a.gamma, lam0, lam1, a.status);
    else
        hipLaunchKernelGGL((k_points_update<kPTX, kPTY, kPNT, 1>), dim3(tx * ty), dim3(kPNT), lds, a.stream, in, C, D,
                           out, a.nx, a.ny, tx, tx * ty, a.gamma, lam0, lam1, a.status);
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    return hipGetLastError();
}

hipError_t prepare_split_f64() {
    const size_t lds = sizeof(PtTile<kPTX, kPTY>);
    hipError_t e = hipFuncSetAttribute((const void*)k_points_update<kPTX, kPTY, kPNT, 0>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_points_update<kPTX, kPTY, kPNT, 1>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

size_t scratch_bytes_split_f64(int nx, int ny) { return (size_t)nx * ny * 28 * sizeof(double); }

}  // namespace af
