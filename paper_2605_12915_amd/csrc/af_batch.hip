// Batching form: many FP32 grids of uneven sizes stepped by ONE launch per step.  The work list holds every (instance, tile) pair of the batch; a grid of
// (CUs x resident workgroups) persistent workgroups walks contiguous chunks of it
// (chunks numbered XCD-aware, so a workgroup's neighbours in the list run on the
// same XCD), calling the same fused tile computation as the single-grid kernel,
// with each instance's own size, background, dt and buffers read from a device
// descriptor array.  af_step_batch captures nsteps launches (alternating the ping-
// pong direction) in a hipGraph and replays it.  The tile shape comes from the
// autotuner (af_api.hip), which times every instantiation below on the batch, in
// both grid modes: persistent (the loop above) and direct (one workgroup per item).
#include <hip/hip_runtime.h>

#include "af_batch.h"
#include "af_fused.h"

namespace af {

// One work item.  Kept out of line on purpose: inlined into the persistent loop below,
// the compiler keeps the tile body's constants live across iterations and spills;
// as a call, the body gets the single-grid kernel's register allocation and the
// loop pays only the callee-saved registers of one call per tile.
template <int TX, int TY, int NT, int SCHEME>
__device__ __noinline__ unsigned batch_tile(const BatchInst* __restrict__ inst, int2 it, int parity) {
    extern __shared__ __align__(16) unsigned char smem[];
    auto& L = *reinterpret_cast<FusedTile<float, TX, TY>*>(smem);
    const BatchInst& d = inst[it.x];
    const PlaneView in{{d.S[parity]}}, out{{d.S[parity ^ 1]}};
    unsigned st = 0;
    fused_tile<float, PolPert<float>, TX, TY, NT, SCHEME, true>(L, in, out, d.comp, d.nx, d.ny,
                                                                (it.y % d.tiles_x) * TX, (it.y / d.tiles_x) * TY,
                                                                d.pol, d.lam0, d.lam1, st);
    return st;
}

// SCHEME (TAI 0, RB 1) is one for the whole batch.
template <int TX, int TY, int NT, int SCHEME>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) k_fused_batch(const BatchInst* __restrict__ inst,
                                                    const int2* __restrict__ work, int nwork, int parity,
                                                    unsigned* status) {
    const int G = gridDim.x;
    // XCD-aware chunk number: consecutive chunks go to workgroups on the same XCD
    int b;
    {
        const int xcd = blockIdx.x & 7;
        int base = 0;
        for (int x = 0; x < xcd; ++x) base += (G - x + 7) >> 3;
        b = base + (blockIdx.x >> 3);
    }
    const int chunk = (nwork + G - 1) / G;
    const int w0 = b * chunk, w1 = min(nwork, w0 + chunk);
    unsigned st = 0;
    for (int w = w0; w < w1; ++w) {
        st |= batch_tile<TX, TY, NT, SCHEME>(inst, work[w], parity);
        __syncthreads();          // the next tile reuses the LDS
    }
    if (st) atomicOr(status, st);
}

// Direct grid mode: one workgroup per work item (the hardware dispatcher balances the
// load), tile body inlined exactly as in the single-grid kernel.  Work items are
// numbered XCD-aware: each XCD gets a contiguous run of the list.
template <int TX, int TY, int NT, int MINW, int SCHEME, int RW = 0>
__global__ void __launch_bounds__(NT, MINW) k_fused_batch_direct(const BatchInst* __restrict__ inst,
                                                           const int2* __restrict__ work, int nwork, int parity,
                                                           unsigned* status) {
    extern __shared__ __align__(16) unsigned char smem[];
    auto& L = *reinterpret_cast<FusedTile<float, TX, TY>*>(smem);
    int w;
    {
        const int b = blockIdx.x, xcd = b & 7;
        int base = 0;
        for (int x = 0; x < xcd; ++x) base += (nwork - x + 7) >> 3;
        w = base + (b >> 3);
    }
    const int2 it = work[w];
    const BatchInst& d = inst[it.x];
    const PlaneView in{{d.S[parity]}}, out{{d.S[parity ^ 1]}};
    unsigned st = 0;
    fused_tile<float, PolPert<float>, TX, TY, NT, SCHEME, true, RW, (RW > 0)>(
        L, in, out, d.comp, d.nx, d.ny, (it.y % d.tiles_x) * TX, (it.y / d.tiles_x) * TY, d.pol, d.lam0, d.lam1, st);
    if (st) atomicOr(status, st);
}

// partner -> caller's buffer for every instance (the odd-step tail of a captured sequence).
__global__ void __launch_bounds__(256) k_batch_copy(const BatchInst* inst, int n) {
    for (int q = 0; q < n; ++q) {
        const BatchInst& d = inst[q];
        const size_t N = (size_t)d.nx * d.ny;
        for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < 16 * N; e += (size_t)gridDim.x * blockDim.x)
            d.S[0][e / N][e % N] = d.S[1][e / N][e % N];
    }
}

template <int TX, int TY, int NT, int MINW, int SCHEME, int RW>
static hipError_t launch_cfg_s(bool direct, const BatchInst* inst, const int2* work, int nwork, int parity,
                               unsigned* status, int grid, hipStream_t s) {
    const size_t lds = sizeof(FusedTile<float, TX, TY>);
    if (direct)
        hipLaunchKernelGGL((k_fused_batch_direct<TX, TY, NT, MINW, SCHEME, RW>), dim3(nwork), dim3(NT), lds, s, inst,
                           work, nwork, parity, status);
    else
        hipLaunchKernelGGL((k_fused_batch<TX, TY, NT, SCHEME>), dim3(grid), dim3(NT), lds, s, inst, work, nwork, parity,
                           status);
    return hipGetLastError();
}

template <int TX, int TY, int NT, int MINW = 1, int RW = 0>
static hipError_t launch_cfg(bool direct, int scheme, const BatchInst* inst, const int2* work, int nwork, int parity,
                             unsigned* status, int grid, hipStream_t s) {
    return scheme ? launch_cfg_s<TX, TY, NT, MINW, 1, RW>(direct, inst, work, nwork, parity, status, grid, s)
                  : launch_cfg_s<TX, TY, NT, MINW, 0, RW>(direct, inst, work, nwork, parity, status, grid, s);
}

template <int TX, int TY, int NT, int MINW, int SCHEME, int RW>
static hipError_t occupancy_cfg_s(bool direct, int* blocks_per_cu) {
    const size_t lds = sizeof(FusedTile<float, TX, TY>);
    if (direct)
        return hipFuncSetAttribute((const void*)k_fused_batch_direct<TX, TY, NT, MINW, SCHEME, RW>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipError_t e = hipFuncSetAttribute((const void*)k_fused_batch<TX, TY, NT, SCHEME>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_fused_batch<TX, TY, NT, SCHEME>, NT, lds);
}

template <int TX, int TY, int NT, int MINW = 1, int RW = 0>
static hipError_t occupancy_cfg(bool direct, int scheme, int* blocks_per_cu) {
    return scheme ? occupancy_cfg_s<TX, TY, NT, MINW, 1, RW>(direct, blocks_per_cu)
                  : occupancy_cfg_s<TX, TY, NT, MINW, 0, RW>(direct, blocks_per_cu);
}

// Candidates: six tile shapes in the persistent mode, the same six direct, 32x8 and
// 24x13 direct with registers capped for 4 waves per SIMD (two workgroups per CU), and
// 31x10 direct, capped, with the targets in rows of 32 lanes and the run-time family
// (the single-grid FP32 kernel's configuration).
const BatchTileCfg kBatchCfgs[kNumBatchCfgs] = {
    {32, 8, 512, false, 1, 0}, {32, 8, 256, false, 1, 0}, {32, 16, 512, false, 1, 0}, {32, 16, 256, false, 1, 0},
    {64, 8, 512, false, 1, 0}, {16, 16, 256, false, 1, 0}, {32, 8, 512, true, 1, 0},   {32, 8, 256, true, 1, 0},
    {32, 16, 512, true, 1, 0}, {32, 16, 256, true, 1, 0},  {64, 8, 512, true, 1, 0},   {16, 16, 256, true, 1, 0},
    {32, 8, 512, true, 4, 0},  {24, 13, 512, true, 4, 0},  {31, 10, 512, true, 4, 32},
};

#define AF_BATCH_SWITCH(F, ...)                                   \
    {                                                             \
        if (cfg == 12) return F<32, 8, 512, 4>(true, __VA_ARGS__); \
        if (cfg == 13) return F<24, 13, 512, 4>(true, __VA_ARGS__); \
        if (cfg == 14) return F<31, 10, 512, 4, 32>(true, __VA_ARGS__); \
        const bool direct = cfg >= 6;                             \
        switch (cfg % 6) {                                        \
            case 0: return F<32, 8, 512>(direct, __VA_ARGS__);    \
            case 1: return F<32, 8, 256>(direct, __VA_ARGS__);    \
            case 2: return F<32, 16, 512>(direct, __VA_ARGS__);   \
            case 3: return F<32, 16, 256>(direct, __VA_ARGS__);   \
            case 4: return F<64, 8, 512>(direct, __VA_ARGS__);    \
            default: return F<16, 16, 256>(direct, __VA_ARGS__);  \
        }                                                         \
    }

hipError_t batch_occupancy(int cfg, int scheme, int* blocks_per_cu) {
    *blocks_per_cu = 1;
    AF_BATCH_SWITCH(occupancy_cfg, scheme, blocks_per_cu)
}

hipError_t launch_batch(int cfg, int scheme, const BatchInst* inst, const int2* work, int nwork, int parity,
                        unsigned* status, int grid, hipStream_t s) {
    AF_BATCH_SWITCH(launch_cfg, scheme, inst, work, nwork, parity, status, grid, s)
}

#undef AF_BATCH_SWITCH

hipError_t launch_batch_copy(const BatchInst* inst, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_copy, dim3(1024), dim3(256), 0, s, inst, n);
    return hipGetLastError();
}

}  // namespace af
