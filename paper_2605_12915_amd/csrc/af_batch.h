// Host/device interface of the batched persistent step (af_batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "af_device.h"

namespace af {

// One grid of a batch: its two state buffers (S[0] = the caller's, S[1] = the
// library's ping-pong partner), Kahan compensation planes, size, background policy
// and dt.
struct BatchInst {
    float* S[2][16];
    float* comp;
    int nx, ny, tiles_x, ntiles;
    PolPert<float> pol;
    float lam0, lam1;
};

// Background policy of the FP32 perturbation form (shared with the single-grid path so
// that both round the background identically).
PolPert<float> pert_pol_f32(const double bg[4], double gamma);

// Plane pointers read from a descriptor in global memory where they are used, as
// global-address-space pointers (plain pointers loaded from memory would otherwise
// be accessed with flat instructions).
using gfloat = __attribute__((address_space(1))) float;
struct PlaneView {
    struct Planes {
        float* const* __restrict__ q;
        __device__ __forceinline__ gfloat* operator[](int k) const { return (gfloat*)q[k]; }
    } p;
};

// rw: point-update targets in rows of rw lanes with the family a run-time value
// (0: tight rows, family a template constant), as in the single-grid kernels
struct BatchTileCfg { int tx, ty, nt; bool direct; int minw; int rw; };
constexpr int kNumBatchCfgs = 15;
extern const BatchTileCfg kBatchCfgs[kNumBatchCfgs];

// scheme: 0 transported (TAI), 1 additive (RB) point update, for the whole batch
hipError_t batch_occupancy(int cfg, int scheme, int* blocks_per_cu);
hipError_t launch_batch(int cfg, int scheme, const BatchInst* inst, const int2* work, int nwork, int parity,
                        unsigned* status, int grid, hipStream_t s);
hipError_t launch_batch_copy(const BatchInst* inst, int n, hipStream_t s);

}  // namespace af
