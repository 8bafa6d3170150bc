// Fused, LDS-tiled RB-TAI step (one launch per step), FP64 and FP32, gfx950.
//
// One workgroup owns a TX x TY tile of cells and produces their new averages and
// the new point values of the nodes they own (V_ij, Ev_ij, Eh_ij).  Every
// intermediate of Sec. 6.1 stays on chip:
//   phase 0  stage the primitive node values of cells [-2, T+3)^2 in LDS,
//   phase 1  recovered centres W^C of cells [-2, T+2)^2 (eq. center-node),
//   phase 2  acoustic increments of V, Ev, Eh, C at node-cells [-1, T+2)^2 for
//            tau = dt/2 and dt (App. D, eq. compact-monomial-block),
//   phase 3  transported point update (Sec. 6.1 steps 3-4) of the targets of
//            node-cells [0, T] (the extra row/column feeds the tile's far edges),
//            and per target the time-Simpson flux (F(W^0) + 4F(W^1/2) + F(W^1))/6,
//   phase 4  spatial Simpson edge fluxes and the average update (eq. af-average-update).
// Halo sizes follow from the foot guard |displacement| < 1 cell: a foot of a target
// in node-cells [0, T] lies in cells [-1, T], whose nodes are node-cells [-1, T+1].
// Workgroups are numbered so that spatially adjacent tiles share an XCD (and its L2).
// The same kernel serves the FP64 path (absolute variables) and the FP32 path
// (perturbations about a background state, PolPert; Kahan-compensated average update
// whose compensation planes persist across steps).
#include <hip/hip_runtime.h>

#include "af_internal.h"
#include "af_kernels.h"

namespace af {

template <class T, int TX, int TY>
struct FusedTile {
    static constexpr int PX = TX + 5, PY = TY + 5;   // primitives: cells [-2, T+3)
    static constexpr int CX = TX + 4, CY = TY + 4;   // centres:    cells [-2, T+2)
    static constexpr int DX = TX + 3, DY = TY + 3;   // increments: node-cells [-1, T+2)
    static constexpr int VX = TX + 1, VY = TY + 1;   // flux nodes: node-cells [0, T]
    T P[12][PY][PX];
    T C[4][CY][CX];
    union {
        T D[2][12][DY][DX];                          // [tau][fam*3 + var]
        struct {
            T FV[8][VY][VX];                         // V nodes: F~ (0..3), G~ (4..7)
            T FE[4][TY][VX];                         // Ev nodes: F~
            T GE[4][VY][TX];                         // Eh nodes: G~
        } F;
    };
};

template <class T, int TX, int TY>
struct LdsAcc {
    const FusedTile<T, TX, TY>* t;
    __device__ __forceinline__ Prim<T> node(int fam, int x, int y) const {
        if (fam == F_C) return {t->C[0][y + 2][x + 2], t->C[1][y + 2][x + 2], t->C[2][y + 2][x + 2], t->C[3][y + 2][x + 2]};
        const int b = 4 * fam;
        return {t->P[b][y + 2][x + 2], t->P[b + 1][y + 2][x + 2], t->P[b + 2][y + 2][x + 2], t->P[b + 3][y + 2][x + 2]};
    }
};

template <class T, int TX, int TY>
struct LdsInc {
    const FusedTile<T, TX, TY>* t;
    int tau;
    __device__ __forceinline__ T inc(int fam, int x, int y, int var) const {
        return t->D[tau][fam * 3 + var][y + 1][x + 1];
    }
};

__device__ __forceinline__ int wrap_any(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <class T, class Pol, int TX, int TY, int NT, int SCHEME, bool KAHAN>
__global__ void __launch_bounds__(NT) k_fused(StatePtrs<T> in, StatePtrs<T> out, T* comp, int nx, int ny,
                                              int tiles_x, int ntiles, Pol pol, T lam0, T lam1, unsigned* status) {
    using Tile = FusedTile<T, TX, TY>;
    extern __shared__ __align__(16) unsigned char smem[];
    Tile& L = *reinterpret_cast<Tile*>(smem);
    const int tid = threadIdx.x;

    // XCD-aware numbering: hardware dispatches consecutive workgroups round-robin over
    // the 8 XCDs; give each XCD a contiguous run of tiles.
    int tile;
    {
        const int b = blockIdx.x, xcd = b & 7;
        int base = 0;
        for (int x = 0; x < xcd; ++x) base += (ntiles - x + 7) >> 3;
        tile = base + (b >> 3);
    }
    const int i0 = (tile % tiles_x) * TX;
    const int j0 = (tile / tiles_x) * TY;
    unsigned st = 0;

    // ---- phase 0: primitive node values of cells [-2, T+3)^2 ------------------------
    for (int e = tid; e < Tile::PX * Tile::PY; e += NT) {
        const int x = e % Tile::PX, y = e / Tile::PX;
        const size_t g = (size_t)wrap_any(j0 + y - 2, ny) * nx + wrap_any(i0 + x - 2, nx);
#pragma unroll
        for (int k = 0; k < 12; ++k) L.P[k][y][x] = in.p[4 + k][g];
    }
    __syncthreads();

    // ---- phase 1: recovered centres of cells [-2, T+2)^2 ------------------------------
    {
        LdsAcc<T, TX, TY> A{&L};
        for (int e = tid; e < Tile::CX * Tile::CY; e += NT) {
            const int x = e % Tile::CX - 2, y = e / Tile::CX - 2;
            const size_t g = (size_t)wrap_any(j0 + y, ny) * nx + wrap_any(i0 + x, nx);
            const T Ub[4] = {in.p[0][g], in.p[1][g], in.p[2][g], in.p[3][g]};
            Prim<T> w = pol.centre(Ub, A.node(F_V, x, y), A.node(F_V, x + 1, y), A.node(F_V, x, y + 1),
                                   A.node(F_V, x + 1, y + 1), A.node(F_EH, x, y), A.node(F_EH, x, y + 1),
                                   A.node(F_EV, x, y), A.node(F_EV, x + 1, y));
            if (!(pol.rho(w.r) > T(0)) || !(pol.pr(w.p) > T(0))) st |= SB_NONPHYS;
            L.C[0][y + 2][x + 2] = w.r;
            L.C[1][y + 2][x + 2] = w.u;
            L.C[2][y + 2][x + 2] = w.v;
            L.C[3][y + 2][x + 2] = w.p;
        }
    }
    __syncthreads();

    // ---- phase 2: increments at node-cells [-1, T+2)^2, both durations ---------------
    {
        LdsAcc<T, TX, TY> A{&L};
        for (int e = tid; e < Tile::DX * Tile::DY; e += NT) {
            const int x = e % Tile::DX - 1, y = e / Tile::DX - 1;
            T d[2][3];
            node_increments<F_V>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][0 * 3 + v][y + 1][x + 1] = d[t][v];
            node_increments<F_EV>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][1 * 3 + v][y + 1][x + 1] = d[t][v];
            node_increments<F_EH>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][2 * 3 + v][y + 1][x + 1] = d[t][v];
            node_increments<F_C>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][3 * 3 + v][y + 1][x + 1] = d[t][v];
        }
    }
    __syncthreads();

    // ---- phase 3: point updates of targets in node-cells [0, T] ----------------------
    constexpr int NV_ = Tile::VX * Tile::VY, NE_ = Tile::VX * TY, NH_ = TX * Tile::VY;
    constexpr int NITEMS = NV_ + NE_ + NH_;
    constexpr int ROUNDS = (NITEMS + NT - 1) / NT;
    T fres[ROUNDS][8];
    {
        LdsAcc<T, TX, TY> A{&L};
        LdsInc<T, TX, TY> D0{&L, 0}, D1{&L, 1};
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int e = r * NT + tid;
            if (e >= NITEMS) continue;
            int fam, x, y;
            if (e < NV_) { fam = F_V; x = e % Tile::VX; y = e / Tile::VX; }
            else if (e < NV_ + NE_) { fam = F_EV; x = (e - NV_) % Tile::VX; y = (e - NV_) / Tile::VX; }
            else { fam = F_EH; x = (e - NV_ - NE_) % TX; y = (e - NV_ - NE_) / TX; }
            Prim<T> w0, wh, w1;
            if (fam == F_V) {
                w0 = A.node(F_V, x, y);
                point_update_pair<F_V, SCHEME>(A, D0, D1, x, y, pol, lam0, lam1, st, wh, w1);
            } else if (fam == F_EV) {
                w0 = A.node(F_EV, x, y);
                point_update_pair<F_EV, SCHEME>(A, D0, D1, x, y, pol, lam0, lam1, st, wh, w1);
            } else {
                w0 = A.node(F_EH, x, y);
                point_update_pair<F_EH, SCHEME>(A, D0, D1, x, y, pol, lam0, lam1, st, wh, w1);
            }
            // new point values of owned nodes
            if (x < TX && y < TY && i0 + x < nx && j0 + y < ny) {
                const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
                const int b = 4 + 4 * fam;
                out.p[b][g] = w1.r;
                out.p[b + 1][g] = w1.u;
                out.p[b + 2][g] = w1.v;
                out.p[b + 3][g] = w1.p;
            }
            T F0[4], Fh[4], F1[4];
            if (fam != F_EH) {
                pol.fx(w0, F0); pol.fx(wh, Fh); pol.fx(w1, F1);
#pragma unroll
                for (int k = 0; k < 4; ++k) fres[r][k] = (F0[k] + T(4) * Fh[k] + F1[k]) * T(1.0 / 6.0);
            }
            if (fam != F_EV) {
                pol.fy(w0, F0); pol.fy(wh, Fh); pol.fy(w1, F1);
                const int o = (fam == F_V) ? 4 : 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) fres[r][o + k] = (F0[k] + T(4) * Fh[k] + F1[k]) * T(1.0 / 6.0);
            }
        }
    }
    __syncthreads();     // every read of D is done: the flux arrays may alias it
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int e = r * NT + tid;
        if (e >= NITEMS) continue;
        if (e < NV_) {
            const int x = e % Tile::VX, y = e / Tile::VX;
#pragma unroll
            for (int k = 0; k < 8; ++k) L.F.FV[k][y][x] = fres[r][k];
        } else if (e < NV_ + NE_) {
            const int x = (e - NV_) % Tile::VX, y = (e - NV_) / Tile::VX;
#pragma unroll
            for (int k = 0; k < 4; ++k) L.F.FE[k][y][x] = fres[r][k];
        } else {
            const int x = (e - NV_ - NE_) % TX, y = (e - NV_ - NE_) / TX;
#pragma unroll
            for (int k = 0; k < 4; ++k) L.F.GE[k][y][x] = fres[r][k];
        }
    }
    __syncthreads();

    // ---- phase 4: average update of the owned cells -----------------------------------
    for (int e = tid; e < TX * TY; e += NT) {
        const int x = e % TX, y = e / TX;
        if (i0 + x >= nx || j0 + y >= ny) continue;
        const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T Fl = (L.F.FV[k][y][x] + T(4) * L.F.FE[k][y][x] + L.F.FV[k][y + 1][x]) * T(1.0 / 6.0);
            const T Fr = (L.F.FV[k][y][x + 1] + T(4) * L.F.FE[k][y][x + 1] + L.F.FV[k][y + 1][x + 1]) * T(1.0 / 6.0);
            const T Gb = (L.F.FV[4 + k][y][x] + T(4) * L.F.GE[k][y][x] + L.F.FV[4 + k][y][x + 1]) * T(1.0 / 6.0);
            const T Gt = (L.F.FV[4 + k][y + 1][x] + T(4) * L.F.GE[k][y + 1][x] + L.F.FV[4 + k][y + 1][x + 1]) * T(1.0 / 6.0);
            const T delta = -lam1 * ((Fr - Fl) + (Gt - Gb));
            if constexpr (KAHAN) {
                // compensated sum: the low-order part lost when adding delta is carried
                // in comp and fed back into the next step's increment
                const size_t N = (size_t)nx * ny;
                const T old = in.p[k][g];
                const T y_ = delta - comp[k * N + g];
                const T t_ = old + y_;
                comp[k * N + g] = (t_ - old) - y_;
                out.p[k][g] = t_;
            } else {
                out.p[k][g] = in.p[k][g] + delta;
            }
        }
    }
    if (st) atomicOr(status, st);
}

constexpr int kTX = 32, kTY = 8, kNT = 512;          // FP64 tile
constexpr int kFTX = 32, kFTY = 8, kFNT = 512;       // FP32 tile

template <class T, class Pol, int TX, int TY, int NT, bool KAHAN>
hipError_t launch_fused(const StepArgs& a, const Pol& pol) {
    StatePtrs<T> in, out;
    for (int k = 0; k < 16; ++k) { in.p[k] = (T*)a.in[k]; out.p[k] = (T*)a.out[k]; }
    const int tiles_x = (a.nx + TX - 1) / TX, tiles_y = (a.ny + TY - 1) / TY;
    const int ntiles = tiles_x * tiles_y;
    const T lam1 = T(a.dt / a.h), lam0 = T(0.5 * a.dt / a.h);
    const size_t lds = sizeof(FusedTile<T, TX, TY>);
    T* comp = (T*)a.comp;
    if (a.ev_begin) (void)hipEventRecord(a.ev_begin, a.stream);
    if (a.scheme == 0)
        hipLaunchKernelGGL((k_fused<T, Pol, TX, TY, NT, 0, KAHAN>), dim3(ntiles), dim3(NT), lds, a.stream, in, out, comp,
                           a.nx, a.ny, tiles_x, ntiles, pol, lam0, lam1, a.status);
    else
        hipLaunchKernelGGL((k_fused<T, Pol, TX, TY, NT, 1, KAHAN>), dim3(ntiles), dim3(NT), lds, a.stream, in, out, comp,
                           a.nx, a.ny, tiles_x, ntiles, pol, lam0, lam1, a.status);
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    return hipGetLastError();
}

template <class T, class Pol, int TX, int TY, int NT, bool KAHAN>
hipError_t prepare_fused() {
    const size_t lds = sizeof(FusedTile<T, TX, TY>);
    hipError_t e = hipFuncSetAttribute((const void*)k_fused<T, Pol, TX, TY, NT, 0, KAHAN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_fused<T, Pol, TX, TY, NT, 1, KAHAN>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_step_fused_f64(const StepArgs& a) {
    PolAbs<double> pol{a.gamma, 1.0 / (a.gamma - 1.0)};
    return launch_fused<double, PolAbs<double>, kTX, kTY, kNT, false>(a, pol);
}

hipError_t prepare_fused_f64() { return prepare_fused<double, PolAbs<double>, kTX, kTY, kNT, false>(); }

PolPert<float> make_pol_f32(const StepArgs& a) {
    const double r0 = a.bg[0], u0 = a.bg[1], v0 = a.bg[2], p0 = a.bg[3], g = a.gamma;
    const double E0 = p0 / (g - 1.0) + 0.5 * r0 * (u0 * u0 + v0 * v0);
    PolPert<float> pol;
    pol.gamma = (float)g;
    pol.gm1inv = (float)(1.0 / (g - 1.0));
    pol.r0 = (float)r0; pol.u0 = (float)u0; pol.v0 = (float)v0; pol.p0 = (float)p0;
    pol.m0x = (float)(r0 * u0); pol.m0y = (float)(r0 * v0); pol.H0 = (float)(E0 + p0);
    return pol;
}

hipError_t launch_step_fused_f32(const StepArgs& a) {
    return launch_fused<float, PolPert<float>, kFTX, kFTY, kFNT, true>(a, make_pol_f32(a));
}

hipError_t prepare_fused_f32() { return prepare_fused<float, PolPert<float>, kFTX, kFTY, kFNT, true>(); }

size_t fused_lds_bytes() { return sizeof(FusedTile<double, kTX, kTY>); }

}  // namespace af
