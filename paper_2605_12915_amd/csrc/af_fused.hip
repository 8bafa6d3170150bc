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
// The kernel template (af_fused.h) serves the FP64 path (absolute variables, this
// file) and the FP32 path (perturbations about a background state, PolPert;
// Kahan-compensated average update whose compensation planes persist across steps;
// af_fused_f32.hip).
#include <hip/hip_runtime.h>

#include "af_fused.h"

namespace af {

// 31x10 cells, 512 threads (154 KB of LDS, one workgroup per CU).  Row stride of the
// staged arrays 36 words; phase 2 has 34x13 = 442 node-cells (one round) and phase 3
// places every target family in rows of 32 lanes: 32x11 V, 32x10 Ev and 31(+1)x11 Eh
// targets fill exactly two rounds of 512, and a half-wavefront (the lanes the LDS
// serves together) reads one row of 32 consecutive doubles (all 64 banks).  The family is a run-time value
// in phase 3 (DYN), so the two wavefronts that hold targets of two families run one
// instruction stream.  Measured at 2048^2 against the earlier 26x12 tile with tight
// item rows and the family as a template constant (1.030 ms): the run-time family
// alone 0.968 ms, the 31x10 rows alone 1.011 ms, both 0.963 ms.
constexpr int kTX = 31, kTY = 10, kNT = 512, kRW = 32;

hipError_t launch_step_fused_f64(const StepArgs& a) {
    PolAbs<double> pol{a.gamma, 1.0 / (a.gamma - 1.0)};
    return launch_fused<double, PolAbs<double>, kTX, kTY, kNT, false, 1, kRW, true>(a, pol);
}

hipError_t prepare_fused_f64() { return prepare_fused<double, PolAbs<double>, kTX, kTY, kNT, false, 1, kRW, true>(); }

size_t fused_lds_bytes() { return sizeof(FusedTile<double, kTX, kTY>); }

}  // namespace af
