// Internal host/device interface between the C ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace af {

// SB_FOOTPRINT: the foot-centred update's disk leaves the half-cell footprint.
enum StatusBits { SB_CFL = 1, SB_FOOT = 2, SB_NONPHYS = 4, SB_FOOTPRINT = 8 };

template <class T>
struct StatePtrs { T* p[16]; };

struct StepArgs {
    int nx, ny;
    double h, gamma, dt;
    int scheme;                 // 0: transported increments, 1: additive RB
    void* in[16];
    void* out[16];
    void* scratch;              // path-specific device scratch
    unsigned* status;           // device status bits (atomicOr)
    hipStream_t stream;
    hipEvent_t ev_begin, ev_end;  // optional: recorded around the dominant kernel
    int variant;                // kernel variant (path-specific)
    double bg[4];               // FP32 path: background (rho, u, v, p) of the perturbations
    void* comp;                 // FP32 path: 4 compensation planes of the average update
};

// Diagnostics partials: 11 values per block (5 sums, min rho, min p, max(|u|+c),
// max c, and two more sums: the vorticity integral and the enstrophy), reduced by
// launch_diag_final.
constexpr int kDiagVals = 11;
// Background of an FP32 state (zeros for FP64): absolute = stored + bg (points),
// stored + Ubg (averages).
struct DiagBg { double bg[4], Ubg[4], gamma; };
DiagBg diag_bg(bool f32, const double bg[4], double gamma);
hipError_t launch_diag_final(const double* partials, int n, double* out9, hipStream_t stream);

hipError_t launch_step_multi_f64(const StepArgs& a);
// Foot-centred exact point update (App. C) in the multi-kernel path; a.scratch holds
// scratch_bytes_fc_f64 bytes.
hipError_t launch_step_fc_f64(const StepArgs& a);
size_t scratch_bytes_fc_f64(int nx, int ny);
hipError_t launch_adjoint_f64(const StepArgs& a, const void* const cot1[16], void* const cot0[16]);
size_t scratch_bytes_adjoint_f64(int nx, int ny);
// Allocation-free adjoint: the scratch lives in a static device array of fixed size
// (grids of at most kNoallocMaxCells cells); a.scratch and a.status are replaced.
constexpr size_t kNoallocMaxCells = size_t(1) << 16;
constexpr size_t kNoallocBytes = (32 + kNoallocMaxCells * 56) * sizeof(double);
hipError_t launch_adjoint_noalloc(StepArgs a, const void* const cot1[16], void* const cot0[16]);
// The device address of that array on the current device (looked up once per device).
hipError_t noalloc_scratch_ptr(void** out);
hipError_t launch_step_fused_f64(const StepArgs& a);
hipError_t launch_step_fused_f32(const StepArgs& a);
hipError_t prepare_fused_f32();
hipError_t prepare_fused_f64();
hipError_t prepare_adjoint_f64();
size_t fused_lds_bytes();
hipError_t launch_step_split_f64(const StepArgs& a);
hipError_t prepare_split_f64();
size_t scratch_bytes_split_f64(int nx, int ny);
size_t scratch_bytes_multi_f64(int nx, int ny);

// Zero `bytes` (a multiple of 8) at device pointer p with a fill kernel on stream s.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

hipError_t launch_diag(const void* const s[16], bool f32, const double bg[4], int nx, int ny, double h,
                       double gamma, double* partials, int npartials, double* out9, hipStream_t stream);

}  // namespace af
