// FP32 precision form of the fused step: float perturbations about a background
// state (PolPert) with the Kahan-compensated average update.  Compiled with
// -ffp-contract=on, like the batched kernel (af_batch.hip): only products and sums
// inside one source expression are fused, so both kernels round every node's
// arithmetic identically and a batched grid reproduces its single-grid result bit
// for bit.
#include <hip/hip_runtime.h>

#include "af_batch.h"
#include "af_fused.h"

namespace af {

// 31x10 cells, 512 threads, registers capped for 4 waves per SIMD (two 77 KB workgroups
// share a CU and overlap each other's barriers), point-update targets in rows of 32
// lanes with the run-time family, as in the FP64 kernel.  Measured at 4096^2 against
// the earlier 24x13 tile with tight rows and the family as a template constant
// (2.061 ms): the run-time family alone 1.994 ms, the 31x10 rows with the constant
// family 1.953 ms, both 1.905 ms; all four give identical bits.  Then the phase-2
// family fence (no more scratch traffic from spills) 1.826 ms and the FP64 row layout
// of the staged arrays (bank conflicts cut eightfold) 1.742 ms, identical bits.
constexpr int kFTX = 31, kFTY = 10, kFNT = 512, kFMinW = 4, kFRW = 32;

PolPert<float> pert_pol_f32(const double bg[4], double g) {
    const double r0 = bg[0], u0 = bg[1], v0 = bg[2], p0 = bg[3];
    const double E0 = p0 / (g - 1.0) + 0.5 * r0 * (u0 * u0 + v0 * v0);
    PolPert<float> pol;
    pol.gamma = (float)g;
    pol.gm1inv = (float)(1.0 / (g - 1.0));
    pol.r0 = (float)r0; pol.u0 = (float)u0; pol.v0 = (float)v0; pol.p0 = (float)p0;
    pol.m0x = (float)(r0 * u0); pol.m0y = (float)(r0 * v0); pol.H0 = (float)(E0 + p0);
    return pol;
}

hipError_t launch_step_fused_f32(const StepArgs& a) {
    return launch_fused<float, PolPert<float>, kFTX, kFTY, kFNT, true, kFMinW, kFRW, true>(a, pert_pol_f32(a.bg, a.gamma));
}

hipError_t prepare_fused_f32() {
    return prepare_fused<float, PolPert<float>, kFTX, kFTY, kFNT, true, kFMinW, kFRW, true>();
}

}  // namespace af
