// The fused, LDS-tiled RB-TAI tile computation (device code shared by the
// single-grid kernel in af_fused.hip and the batched persistent kernel in
// af_batch.hip).  See af_fused.hip for the phase structure.
#pragma once
#include <hip/hip_runtime.h>

#include "af_internal.h"
#include "af_kernels.h"
#include "af_tile.h"

namespace af {

template <int B, class SP, class T>
__device__ __forceinline__ void store_prim(const SP& o, size_t g, const Prim<T>& w) {
    o.p[B][g] = w.r;
    o.p[B + 1][g] = w.u;
    o.p[B + 2][g] = w.v;
    o.p[B + 3][g] = w.p;
}

// One tile: cells [i0, i0+TX) x [j0, j0+TY) of one grid.  Called by the single-grid
// kernel (one tile per workgroup) and by the batched persistent kernel (a list of
// tiles of many grids per workgroup).  The arithmetic of every node does not depend
// on the tile shape or on which kernel calls it; compiled with -ffp-contract=on in
// both, the FP32 kernels therefore agree bit for bit.
// Phase 2 computes the four families' increments one after the other with a
// scheduling fence between them.  Interleaving them (the compiler's choice without it)
// needs more registers than a wave holds at these occupancies and spills: in FP64
// beyond 256, in the FP32 kernels (128 at two workgroups per CU) 14 registers, whose
// scratch traffic reached HBM (1.9x the algorithmic bytes written).
//
// SP: any type with a member p such that p[k] is plane k's pointer (StatePtrs, or a
// view of a descriptor in global memory whose pointers are loaded where used).
// RW: phase 3 lays each target family's items out in rows of RW lanes (0: rows as
// wide as the family's own row of targets).  With RW a multiple of 16, the lanes that
// the LDS serves together read consecutive words of one row (no bank conflicts for
// feet at a common offset).  DYN: the family of a target is a run-time value, so a
// wavefront holding targets of two families runs one instruction stream instead of
// both families' code one after the other.
template <class T, class Pol, int TX, int TY, int NT, int SCHEME, bool KAHAN, int RW = 0, bool DYN = false,
          class SP>
__device__ __forceinline__ void fused_tile(FusedTile<T, TX, TY>& L, const SP& in, const SP& out,
                                           T* comp, int nx, int ny, int i0, int j0, const Pol pol, T lam0, T lam1,
                                           unsigned& st) {
    using Tile = FusedTile<T, TX, TY>;
    const int tid = threadIdx.x;

    // windows reach 2 cells below and 3 above the tile: one wrap suffices when the
    // grid spans the window
    const bool onex = nx >= Tile::PX, oney = ny >= Tile::PY;

    // ---- phase 0: primitive node values of cells [-2, T+3)^2 ------------------------
    if constexpr (sizeof(T) == 8) {
        // every round's loads issued before the first store: the window has slightly more
        // node-cells than threads, and a second load round trip would hold the whole
        // workgroup at the barrier (1.5% faster; in FP32 the extra live registers cost more)
        constexpr int NP0 = Tile::PX * Tile::PY, R0 = (NP0 + NT - 1) / NT;
        T pv[R0][12];
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int e = r * NT + tid;
            int x, y;
            if (Tile::stage_item(e, x, y)) {
                const size_t g = (size_t)wrap_win(j0 + y - 2, ny, oney) * nx + wrap_win(i0 + x - 2, nx, onex);
#pragma unroll
                for (int k = 0; k < 12; ++k) pv[r][k] = in.p[4 + k][g];
            }
        }
#pragma unroll
        for (int r = 0; r < R0; ++r) {
            const int e = r * NT + tid;
            int x, y;
            if (Tile::stage_item(e, x, y))
#pragma unroll
                for (int k = 0; k < 12; ++k) L.P[k][y][x] = pv[r][k];
        }
    } else {
        for (int e = tid; e < Tile::PX * Tile::PY; e += NT) {
            int x, y;
            Tile::stage_item(e, x, y);
            const size_t g = (size_t)wrap_win(j0 + y - 2, ny, oney) * nx + wrap_win(i0 + x - 2, nx, onex);
#pragma unroll
            for (int k = 0; k < 12; ++k) L.P[k][y][x] = in.p[4 + k][g];
        }
    }
    __syncthreads();

    // ---- phase 1: recovered centres of cells [-2, T+2)^2 ------------------------------
    {
        LdsAcc<T, TX, TY> A{&L};
        for (int e = tid; e < Tile::SC * Tile::CY; e += NT) {
            int x, y;
            if (!Tile::centre_item(e, x, y)) continue;
            const size_t g = (size_t)wrap_win(j0 + y, ny, oney) * nx + wrap_win(i0 + x, nx, onex);
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
        for (int e = tid; e < Tile::SD * Tile::DY; e += NT) {
            int x, y;
            if (!Tile::incr_item(e, x, y)) continue;
            T d[2][3];
            node_increments<F_V>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][0 * 3 + v][y + 1][x + 1] = d[t][v];
            __builtin_amdgcn_sched_barrier(0);   // one family at a time
            node_increments<F_EV>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][1 * 3 + v][y + 1][x + 1] = d[t][v];
            __builtin_amdgcn_sched_barrier(0);   // one family at a time
            node_increments<F_EH>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][2 * 3 + v][y + 1][x + 1] = d[t][v];
            __builtin_amdgcn_sched_barrier(0);   // one family at a time
            node_increments<F_C>(A, x, y, pol, lam0, lam1, d, st);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int v = 0; v < 3; ++v) L.D[t][3 * 3 + v][y + 1][x + 1] = d[t][v];
        }
    }
    __syncthreads();

    // ---- phase 3: point updates of targets in node-cells [0, T] ----------------------
    using Pts = typename Tile::template Points<RW>;
    static_assert(Pts::WV >= Tile::VX && Pts::WH >= TX, "item rows hold a row of targets");
    constexpr int NITEMS = Pts::N;
    constexpr int ROUNDS = (NITEMS + NT - 1) / NT;
    T fres[ROUNDS][8];
    {
        LdsAcc<T, TX, TY> A{&L};
        LdsInc<T, TX, TY> D0{&L, 0}, D1{&L, 1};
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const int e = r * NT + tid;
            int fam, x, y;
            if (!Pts::item(e, fam, x, y)) continue;
            Prim<T> w0, wh, w1;
            // new point values of owned nodes (plane indices kept static: a dynamic
            // index into the pointer set would put it in private memory)
            const bool own = x < TX && y < TY && i0 + x < nx && j0 + y < ny;
            const size_t g = own ? (size_t)(j0 + y) * nx + (i0 + x) : 0;
            if constexpr (DYN) {
                w0 = A.node(fam, x, y);
                point_update_pair_f<SCHEME>(A, D0, D1, fam, x, y, pol, lam0, lam1, st, wh, w1);
                if (own) {
                    if (fam == F_V) store_prim<4>(out, g, w1);
                    else if (fam == F_EV) store_prim<8>(out, g, w1);
                    else store_prim<12>(out, g, w1);
                }
            } else if (fam == F_V) {
                w0 = A.node(F_V, x, y);
                point_update_pair<F_V, SCHEME>(A, D0, D1, x, y, pol, lam0, lam1, st, wh, w1);
                if (own) store_prim<4>(out, g, w1);
            } else if (fam == F_EV) {
                w0 = A.node(F_EV, x, y);
                point_update_pair<F_EV, SCHEME>(A, D0, D1, x, y, pol, lam0, lam1, st, wh, w1);
                if (own) store_prim<8>(out, g, w1);
            } else {
                w0 = A.node(F_EH, x, y);
                point_update_pair<F_EH, SCHEME>(A, D0, D1, x, y, pol, lam0, lam1, st, wh, w1);
                if (own) store_prim<12>(out, g, w1);
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
    // FP32: the owned cells' time-n averages and compensation for phase 4 are loaded
    // here, so that their latency overlaps the flux stores and the two barriers (5%
    // faster; in FP64 the registers they hold across the barriers cost 0.7%).
    constexpr bool kEarlyAvg = sizeof(T) == 4;
    constexpr int R4 = (TX * TY + NT - 1) / NT;
    T oldv[R4][4], oldc[R4][4];
    if constexpr (kEarlyAvg) {
#pragma unroll
        for (int r = 0; r < R4; ++r) {
            const int e = r * NT + tid;
            int x, y;
            if (Tile::update_item(e, x, y) && i0 + x < nx && j0 + y < ny) {
                const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
#pragma unroll
                for (int k = 0; k < 4; ++k) oldv[r][k] = in.p[k][g];
                if constexpr (KAHAN) {
                    const size_t N = (size_t)nx * ny;
                    auto* __restrict__ cg = (__attribute__((address_space(1))) T*)comp;
#pragma unroll
                    for (int k = 0; k < 4; ++k) oldc[r][k] = cg[k * N + g];
                }
            }
        }
    }
    __syncthreads();     // every read of D is done: the flux arrays may alias it
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int e = r * NT + tid;
        int fam, x, y;
        if (!Pts::item(e, fam, x, y)) continue;
        if (fam == F_V) {
#pragma unroll
            for (int k = 0; k < 8; ++k) L.F.FV[k][y][x] = fres[r][k];
        } else if (fam == F_EV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) L.F.FE[k][y][x] = fres[r][k];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) L.F.GE[k][y][x] = fres[r][k];
        }
    }
    __syncthreads();

    // ---- phase 4: average update of the owned cells -----------------------------------
    // -lam1 times the divergence of the cell's four space-time Simpson edge fluxes
    auto delta_of = [&](int x, int y, int k) -> T {
        const T Fl = (L.F.FV[k][y][x] + T(4) * L.F.FE[k][y][x] + L.F.FV[k][y + 1][x]) * T(1.0 / 6.0);
        const T Fr = (L.F.FV[k][y][x + 1] + T(4) * L.F.FE[k][y][x + 1] + L.F.FV[k][y + 1][x + 1]) * T(1.0 / 6.0);
        const T Gb = (L.F.FV[4 + k][y][x] + T(4) * L.F.GE[k][y][x] + L.F.FV[4 + k][y][x + 1]) * T(1.0 / 6.0);
        const T Gt = (L.F.FV[4 + k][y + 1][x] + T(4) * L.F.GE[k][y + 1][x] + L.F.FV[4 + k][y + 1][x + 1]) * T(1.0 / 6.0);
        return -lam1 * ((Fr - Fl) + (Gt - Gb));
    };
    if constexpr (kEarlyAvg) {
#pragma unroll
        for (int r = 0; r < R4; ++r) {
            const int e = r * NT + tid;
            int x, y;
            if (!Tile::update_item(e, x, y)) continue;
            if (i0 + x >= nx || j0 + y >= ny) continue;
            const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T delta = delta_of(x, y, k);
                if constexpr (KAHAN) {
                    // compensated sum: the low-order part lost when adding delta is carried
                    // in comp and fed back into the next step's increment
                    const size_t N = (size_t)nx * ny;
                    auto* __restrict__ cg = (__attribute__((address_space(1))) T*)comp;
                    const T old = oldv[r][k];
                    const T y_ = delta - oldc[r][k];
                    const T t_ = old + y_;
                    cg[k * N + g] = (t_ - old) - y_;
                    out.p[k][g] = t_;
                } else {
                    out.p[k][g] = oldv[r][k] + delta;
                }
            }
        }
    } else {
        for (int e = tid; e < TX * TY; e += NT) {
            int x, y;
            Tile::update_item(e, x, y);
            if (i0 + x >= nx || j0 + y >= ny) continue;
            const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T delta = delta_of(x, y, k);
                if constexpr (KAHAN) {
                    const size_t N = (size_t)nx * ny;
                    auto* __restrict__ cg = (__attribute__((address_space(1))) T*)comp;
                    const T old = in.p[k][g];
                    const T y_ = delta - cg[k * N + g];
                    const T t_ = old + y_;
                    cg[k * N + g] = (t_ - old) - y_;
                    out.p[k][g] = t_;
                } else {
                    out.p[k][g] = in.p[k][g] + delta;
                }
            }
        }
    }
}

// ---- single-grid kernel: one tile per workgroup --------------------------------------
// MINW: minimum wavefronts per SIMD the register allocation must allow (1: no
// constraint beyond the workgroup size; 4 at 512 threads: two workgroups per CU).
template <class T, class Pol, int TX, int TY, int NT, int SCHEME, bool KAHAN, int MINW = 1, int RW = 0,
          bool DYN = false>
__global__ void __launch_bounds__(NT, MINW) k_fused(StatePtrs<T> in, StatePtrs<T> out, T* comp, int nx, int ny,
                                              int tiles_x, int ntiles, Pol pol, T lam0, T lam1, unsigned* status) {
    extern __shared__ __align__(16) unsigned char smem[];
    auto& L = *reinterpret_cast<FusedTile<T, TX, TY>*>(smem);
    // XCD-aware numbering: hardware dispatches consecutive workgroups round-robin over
    // the 8 XCDs; give each XCD a contiguous run of tiles.
    int tile;
    {
        const int b = blockIdx.x, xcd = b & 7;
        int base = 0;
        for (int x = 0; x < xcd; ++x) base += (ntiles - x + 7) >> 3;
        tile = base + (b >> 3);
    }
    unsigned st = 0;
    fused_tile<T, Pol, TX, TY, NT, SCHEME, KAHAN, RW, DYN>(L, in, out, comp, nx, ny, (tile % tiles_x) * TX,
                                                           (tile / tiles_x) * TY, pol, lam0, lam1, st);
    if (st) atomicOr(status, st);
}


template <class T, class Pol, int TX, int TY, int NT, bool KAHAN, int MINW = 1, int RW = 0, bool DYN = false>
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
        hipLaunchKernelGGL((k_fused<T, Pol, TX, TY, NT, 0, KAHAN, MINW, RW, DYN>), dim3(ntiles), dim3(NT), lds, a.stream, in, out, comp,
                           a.nx, a.ny, tiles_x, ntiles, pol, lam0, lam1, a.status);
    else
        hipLaunchKernelGGL((k_fused<T, Pol, TX, TY, NT, 1, KAHAN, MINW, RW, DYN>), dim3(ntiles), dim3(NT), lds, a.stream, in, out, comp,
                           a.nx, a.ny, tiles_x, ntiles, pol, lam0, lam1, a.status);
    if (a.ev_end) (void)hipEventRecord(a.ev_end, a.stream);
    return hipGetLastError();
}

template <class T, class Pol, int TX, int TY, int NT, bool KAHAN, int MINW = 1, int RW = 0, bool DYN = false>
hipError_t prepare_fused() {
    const size_t lds = sizeof(FusedTile<T, TX, TY>);
    hipError_t e = hipFuncSetAttribute((const void*)k_fused<T, Pol, TX, TY, NT, 0, KAHAN, MINW, RW, DYN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_fused<T, Pol, TX, TY, NT, 1, KAHAN, MINW, RW, DYN>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace af
