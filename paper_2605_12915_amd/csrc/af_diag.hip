// FP64 diagnostics of a state (Sec. 6 opening paragraph: CFL and the entropy
// functional -int rho log(p / rho^gamma) dA; Sec. 3: conservation totals; Sec. 6,
// low-Mach shear: the integrals of the vorticity and of its square, for the
// continuous piecewise-Q2 velocity reconstruction).
// Two passes: a grid-stride block reduction into per-block partials (wavefront
// shuffles, then LDS across the block's wavefronts), then one block over the
// partials.  Entropy uses the tensor Simpson rule over the nine Q2 nodes of a cell
// (the recovered centre included), regrouped per node.
#include <hip/hip_runtime.h>

#include "af_internal.h"
#include "af_kernels.h"
#include "af_reduce.h"

namespace af {

constexpr int kDiagBlock = 256;


__device__ __forceinline__ void block_reduce(double v[kDiagVals], double* sh) {
    diag_wave_reduce(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kDiagVals; ++k) sh[wid * kDiagVals + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) diag_combine(v, sh + w * kDiagVals);
    }
}

// Reads a state of T (absolute doubles, or float perturbations about bg) as
// absolute FP64 values.
template <class T>
struct DiagAcc {
    const T* s[16];
    int nx, ny;
    double gamma;
    double bg[4], Ubg[4];
    __device__ __forceinline__ double val(int plane, size_t k) const {
        const int b = plane < 4 ? -1 : (plane - 4) % 4;
        return (double)s[plane][k] + (plane < 4 ? Ubg[plane] : bg[b]);
    }
    __device__ __forceinline__ size_t idx(int i, int j) const {
        i = i >= nx ? i - nx : i;
        j = j >= ny ? j - ny : j;
        return (size_t)j * nx + i;
    }
    __device__ __forceinline__ Prim<double> point(int fam, int i, int j) const {
        const size_t k = idx(i, j);
        const int b = 4 + 4 * fam;
        return {val(b, k), val(b + 1, k), val(b + 2, k), val(b + 3, k)};
    }
    // (not recursive, so that it inlines: a call would spill the whole state)
    __device__ __forceinline__ Prim<double> node(int fam, int i, int j) const {
        if (fam == F_C) {
            const size_t k = idx(i, j);
            double Ub[4] = {val(0, k), val(1, k), val(2, k), val(3, k)};
            return recover_centre(Ub, point(F_V, i, j), point(F_V, i + 1, j), point(F_V, i, j + 1),
                                  point(F_V, i + 1, j + 1), point(F_EH, i, j), point(F_EH, i, j + 1),
                                  point(F_EV, i, j), point(F_EV, i + 1, j), gamma);
        }
        return point(fam, i, j);
    }
};

// Two waves per SIMD (181 registers, no spill).  With the logarithm of af_math.h the
// 4-wave cap that suited the library's logarithm (5 dwords spilled then, 0.29 ms per call
// at 2048^2) spills 56 dwords (0.73 ms) and a 3-wave cap 14 (0.30 ms); 0.23 ms here.
template <class T>
__global__ void __launch_bounds__(kDiagBlock, 2) k_diag(StatePtrs<const T> st, int nx, int ny, double gamma,
                                                     DiagBg bgs, double* partials) {
    __shared__ double sh[(kDiagBlock / 64) * kDiagVals];
    DiagAcc<T> A;
    A.nx = nx;
    A.ny = ny;
    A.gamma = gamma;
#pragma unroll
    for (int k = 0; k < 4; ++k) { A.bg[k] = bgs.bg[k]; A.Ubg[k] = bgs.Ubg[k]; }
#pragma unroll
    for (int k = 0; k < 16; ++k) A.s[k] = st.p[k];
    double v[kDiagVals];
    diag_init(v);
    const size_t N = (size_t)nx * ny;
    // Entropy: the tensor Simpson rule over the nine Q2 nodes of every cell, summed
    // over cells, gives each node the sum of its weights in the cells that share it:
    // vertex 4 x 1/36 = 1/9, edge midpoints 2 x 4/36 = 2/9, centre 16/36 = 4/9.  So
    // each cell evaluates its own four nodes (V, Ev, Eh, C) once.
    const double wnode[4] = {kWNodeV, kWNodeE, kWNodeE, kWNodeC};
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += stride) {
        // 32-bit division when the grid allows (64-bit division costs ~10x more)
        int i, j;
        if (N <= 0xffffffffull) {
            const unsigned cu = (unsigned)c, nxu = (unsigned)nx;
            j = (int)(cu / nxu);
            i = (int)(cu - (unsigned)j * nxu);
        } else {
            i = (int)(c % nx);
            j = (int)(c / nx);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += A.val(k, c);
        const Prim<double> own[4] = {A.point(F_V, i, j), A.point(F_EV, i, j), A.point(F_EH, i, j), A.node(F_C, i, j)};
#pragma unroll
        for (int f = 0; f < 4; ++f) diag_node(v, wnode[f], own[f].r, own[f].u, own[f].v, own[f].p, gamma);
        // the cell's nine velocity nodes, [x-node][y-node]
        const Prim<double> v10 = A.point(F_V, i + 1, j), v01 = A.point(F_V, i, j + 1), v11 = A.point(F_V, i + 1, j + 1);
        const Prim<double> ev1 = A.point(F_EV, i + 1, j), eh1 = A.point(F_EH, i, j + 1);
        const double cu[3][3] = {{own[0].u, own[1].u, v01.u}, {own[2].u, own[3].u, eh1.u}, {v10.u, ev1.u, v11.u}};
        const double cv[3][3] = {{own[0].v, own[1].v, v01.v}, {own[2].v, own[3].v, eh1.v}, {v10.v, ev1.v, v11.v}};
        diag_vorticity(v, cu, cv);
    }
    block_reduce(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < kDiagVals; ++k) partials[(size_t)blockIdx.x * kDiagVals + k] = v[k];
}

__global__ void __launch_bounds__(kDiagBlock) k_diag_final(const double* partials, int n, double* out) {
    __shared__ double sh[(kDiagBlock / 64) * kDiagVals];
    double v[kDiagVals];
    diag_init(v);
    for (int b = threadIdx.x; b < n; b += blockDim.x) diag_combine(v, partials + (size_t)b * kDiagVals);
    block_reduce(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < kDiagVals; ++k) out[k] = v[k];
}

DiagBg diag_bg(bool f32, const double bg[4], double gamma) {
    DiagBg b;
    b.gamma = gamma;
    for (int k = 0; k < 4; ++k) { b.bg[k] = f32 ? bg[k] : 0.0; b.Ubg[k] = 0.0; }
    if (f32) {
        b.Ubg[0] = bg[0];
        b.Ubg[1] = bg[0] * bg[1];
        b.Ubg[2] = bg[0] * bg[2];
        b.Ubg[3] = bg[3] / (gamma - 1.0) + 0.5 * bg[0] * (bg[1] * bg[1] + bg[2] * bg[2]);
    }
    return b;
}

hipError_t launch_diag_final(const double* partials, int n, double* out9, hipStream_t stream) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagBlock), 0, stream, partials, n, out9);
    return hipGetLastError();
}

hipError_t launch_diag(const void* const s[16], bool f32, const double bg[4], int nx, int ny, double h,
                       double gamma, double* partials, int npartials, double* out9, hipStream_t stream) {
    const DiagBg b = diag_bg(f32, bg, gamma);
    if (f32) {
        StatePtrs<const float> st;
        for (int k = 0; k < 16; ++k) st.p[k] = (const float*)s[k];
        hipLaunchKernelGGL(k_diag<float>, dim3(npartials), dim3(kDiagBlock), 0, stream, st, nx, ny, gamma, b, partials);
    } else {
        StatePtrs<const double> st;
        for (int k = 0; k < 16; ++k) st.p[k] = (const double*)s[k];
        hipLaunchKernelGGL(k_diag<double>, dim3(npartials), dim3(kDiagBlock), 0, stream, st, nx, ny, gamma, b, partials);
    }
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kDiagBlock), 0, stream, partials, npartials, out9);
    return hipGetLastError();
}

}  // namespace af
