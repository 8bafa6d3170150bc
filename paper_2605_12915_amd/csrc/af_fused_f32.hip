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

// 24x13 cells, 512 threads, registers capped for 4 waves per SIMD: two 74 KB workgroups
// share a CU (a 32x8 tile with the same cap was 12% faster than one 32x16 workgroup
// with free register allocation; 24x13 fills the increment and point phases' rounds
// of 512 threads better than 32x8 and is 4.6% faster again).
constexpr int kFTX = 24, kFTY = 13, kFNT = 512, kFMinW = 4;

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
    return launch_fused<float, PolPert<float>, kFTX, kFTY, kFNT, true, kFMinW>(a, pert_pol_f32(a.bg, a.gamma));
}

hipError_t prepare_fused_f32() { return prepare_fused<float, PolPert<float>, kFTX, kFTY, kFNT, true, kFMinW>(); }

}  // namespace af
