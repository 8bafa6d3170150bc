// Device building blocks of the RB-TAI Active Flux step for gfx950 (FP64 and FP32).
//
// Every function here is a small, fully inlined piece of the algorithm of Sec. 6.1:
//   centre recovery from the conservative Simpson constraint (eq. center-node),
//   the node-centred exact acoustic operator in compact monomial-block form
//   (App. D, eq. compact-monomial-block), the Q2 evaluation used for the convective
//   foot and for the increment interpolant (Sec. 4, R_Delta), the transported point
//   update (Sec. 6.1 steps 3-4) and the Euler fluxes (Sec. 3).
// Data access goes through an accessor type (global planes or an LDS tile) so that
// the multi-kernel and the fused kernels share the arithmetic.
#pragma once
#include <hip/hip_runtime.h>

#include "af_blocks.h"
#include "af_internal.h"

// Helpers are host+device so that the operation-counting build (count_flops.cpp)
// can run the very same arithmetic on the host.
#ifndef AF_HD
#define AF_HD __host__ __device__ __forceinline__
#endif

namespace af {

// 1 / sqrt(x): the device's reciprocal square root (one hardware estimate and its
// refinement in FP64, the hardware instruction in FP32); the host builds that check
// indexing and count operations take the plain quotient.
AF_HD double rsqrt_of(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return rsqrt(x);
#else
    return 1.0 / sqrt(x);
#endif
}
AF_HD float rsqrt_of(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return rsqrtf(x);
#else
    return 1.0f / sqrtf(x);
#endif
}

// a / b: the correctly rounded quotient in FP64; in FP32 the product with the hardware
// reciprocal (within 1 ulp; a few instructions against the division's scaled iteration),
// whose rounding is far inside the FP32 form's stated error; the host builds divide.
AF_HD double quot(double a, double b) { return a / b; }
AF_HD float quot(float a, float b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return a * __builtin_amdgcn_rcpf(b);
#else
    return a / b;
#endif
}

enum Fam { F_V = 0, F_EV = 1, F_EH = 2, F_C = 3 };

template <class T>
struct Prim { T r, u, v, p; };

// ---------------------------------------------------------------------------
// Conservative <-> primitive (Sec. 2)
// ---------------------------------------------------------------------------
template <class T>
AF_HD void cons_of(const Prim<T>& w, T gm1inv, T U[4]) {
    U[0] = w.r;
    U[1] = w.r * w.u;
    U[2] = w.r * w.v;
    U[3] = w.p * gm1inv + T(0.5) * w.r * (w.u * w.u + w.v * w.v);
}

// Recovered centre node (eq. center-node), written about the anchor U_a = U(V_ij)
// so that uniform data returns the anchor exactly (free-stream preservation):
//   U_c = U_a + 9/4 [ (Ubar - U_a) - sum_corners (U - U_a)/36 - sum_edges (U - U_a)/9 ].
template <class T>
AF_HD Prim<T> recover_centre(const T Ub[4], const Prim<T>& v00, const Prim<T>& v10,
                                                  const Prim<T>& v01, const Prim<T>& v11, const Prim<T>& eh0,
                                                  const Prim<T>& eh1, const Prim<T>& ev0, const Prim<T>& ev1,
                                                  T gamma) {
    const T gm1inv = T(1) / (gamma - T(1));
    T Ua[4], U[4], sc[4], se[4];
    cons_of(v00, gm1inv, Ua);
    cons_of(v10, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) sc[k] = U[k] - Ua[k];
    cons_of(v01, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) sc[k] += U[k] - Ua[k];
    cons_of(v11, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) sc[k] += U[k] - Ua[k];
    cons_of(eh0, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) se[k] = U[k] - Ua[k];
    cons_of(eh1, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) se[k] += U[k] - Ua[k];
    cons_of(ev0, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) se[k] += U[k] - Ua[k];
    cons_of(ev1, gm1inv, U);
#pragma unroll
    for (int k = 0; k < 4; ++k) se[k] += U[k] - Ua[k];
    T Uc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        Uc[k] = Ua[k] + T(2.25) * ((Ub[k] - Ua[k]) - sc[k] * T(1.0 / 36.0) - se[k] * T(1.0 / 9.0));
    Prim<T> w;
    w.r = Uc[0];
    T ir = T(1) / Uc[0];
    w.u = Uc[1] * ir;
    w.v = Uc[2] * ir;
    w.p = (gamma - T(1)) * (Uc[3] - T(0.5) * (Uc[1] * w.u + Uc[2] * w.v));
    return w;
}

// ---------------------------------------------------------------------------
// Exact node-centred acoustic operator (App. D)
// ---------------------------------------------------------------------------
// Monomial coefficients of the 1-D quadratic through (f0, f1, f2) at X0, X0+1/2,
// X0+1 (units of h), written in differences so that constants give exact zeros.
// XC = 0: X0 = 0;  XC = 1: X0 = -1;  XC = 2: X0 = -1/2.
template <int XC, class T>
AF_HD void mono1(T f0, T f1, T f2, T& c0, T& c1, T& c2) {
    T d10 = f1 - f0, d20 = f2 - f0, d21 = f2 - f1;
    c2 = T(2) * d20 - T(4) * d10;
    if constexpr (XC == 0) { c0 = f0; c1 = T(4) * d10 - d20; }
    else if constexpr (XC == 1) { c0 = f2; c1 = T(4) * d21 - d20; }
    else { c0 = f1; c1 = d20; }
}

// Accumulators of one node: the r^m coefficient (m = 1..4) of
//   [0] p-out from p-in, [1] p-out / Z from (u,v)-in, [2] u-out * Z from p-in,
//   [3] u-out from (u,v)-in, [4] v-out * Z from p-in, [5] v-out from (u,v)-in.
template <class T>
struct NodeAcc {
    T a[6][4];
    AF_HD void zero() {
#pragma unroll
        for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int m = 0; m < 4; ++m) a[c][m] = T(0);
    }
};

// Add the contribution of wedge W (cell nodal data f[var][x-node][y-node] of
// (p, u, v); the cell's lower-left node at (X0, Y0) relative to the node).
template <int W, int XC, int YC, class T>
AF_HD void wedge_acc(const T f[3][3][3], NodeAcc<T>& acc) {
    T c[3][3][3];   // [var][alpha][beta]
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        T g[3][3];  // [alpha][y-node]
#pragma unroll
        for (int b = 0; b < 3; ++b) mono1<XC>(f[v][0][b], f[v][1][b], f[v][2][b], g[0][b], g[1][b], g[2][b]);
#pragma unroll
        for (int al = 0; al < 3; ++al) mono1<YC>(g[al][0], g[al][1], g[al][2], c[v][al][0], c[v][al][1], c[v][al][2]);
    }
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
            if (al + be == 0) continue;
            const int m = al + be - 1;
            const double* B = kBlk[W][al][be];
            const T cp = c[0][al][be], cu = c[1][al][be], cv = c[2][al][be];
            if (B[0] != 0.0) acc.a[0][m] += T(B[0]) * cp;
            if (B[1] != 0.0) acc.a[1][m] += T(B[1]) * cu;
            if (B[2] != 0.0) acc.a[1][m] += T(B[2]) * cv;
            if (B[3] != 0.0) acc.a[2][m] += T(B[3]) * cp;
            if (B[4] != 0.0) acc.a[3][m] += T(B[4]) * cu;
            if (B[5] != 0.0) acc.a[3][m] += T(B[5]) * cv;
            if (B[6] != 0.0) acc.a[4][m] += T(B[6]) * cp;
            if (B[7] != 0.0) acc.a[5][m] += T(B[7]) * cu;
            if (B[8] != 0.0) acc.a[5][m] += T(B[8]) * cv;
        }
}

// Increments (du, dv, dp) at radius r from the accumulators; Z = rho_K c_K.
template <class T>
AF_HD void node_increment(const NodeAcc<T>& A, T r, T Z, T iZ, T inc[3]) {
    T s[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) s[c] = ((A.a[c][3] * r + A.a[c][2]) * r + A.a[c][1]) * r + A.a[c][0];
    inc[0] = r * (s[2] * iZ + s[3]);
    inc[1] = r * (s[4] * iZ + s[5]);
    inc[2] = r * (s[0] + Z * s[1]);
}

// ---------------------------------------------------------------------------
// Q2 evaluation and the transported point update
// ---------------------------------------------------------------------------
// Lagrange weights at -1 and +1 (the middle one is implied by the difference form).
template <class T>
AF_HD void lag_pm(T s, T& lm, T& lp) {
    T hs = T(0.5) * s;
    lm = hs * (s - T(1));
    lp = hs * (s + T(1));
}

// sum_a l_a f_a written as f_1 + l_-(f_0 - f_1) + l_+(f_2 - f_1): exact on constants.
template <class T>
AF_HD T q1(T lm, T lp, T f0, T f1, T f2) {
    return f1 + lm * (f0 - f1) + lp * (f2 - f1);
}

template <class T>
AF_HD T q2(T xm, T xp, T ym, T yp, const T f[3][3]) {
    T g0 = q1(xm, xp, f[0][0], f[1][0], f[2][0]);
    T g1 = q1(xm, xp, f[0][1], f[1][1], f[2][1]);
    T g2 = q1(xm, xp, f[0][2], f[1][2], f[2][2]);
    return q1(ym, yp, g0, g1, g2);
}

// FP32: the tensor weights lx[a] ly[b] (lx = (xm, 1 - xm - xp, xp)) times the nodal values,
// nine products whose weights every evaluation at the same point shares (the compiler
// forms them once), against sixteen operations per evaluation in the difference form.
// The FP32 form's values are perturbations about a uniform background, which stays exact
// (a zero perturbation stays zero); the FP64 path keeps the difference form, exact on
// constants.
template <>
AF_HD float q2<float>(float xm, float xp, float ym, float yp, const float f[3][3]) {
    const float lx[3] = {xm, 1.0f - xm - xp, xp}, ly[3] = {ym, 1.0f - ym - yp, yp};
    float s = 0.0f;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) s += (lx[a] * ly[b]) * f[a][b];
    return s;
}

template <class T>
AF_HD void flux_x(const Prim<T>& w, T gm1inv, T F[4]) {
    T E = w.p * gm1inv + T(0.5) * w.r * (w.u * w.u + w.v * w.v);
    T m = w.r * w.u;
    F[0] = m;
    F[1] = m * w.u + w.p;
    F[2] = m * w.v;
    F[3] = w.u * (E + w.p);
}

template <class T>
AF_HD void flux_y(const Prim<T>& w, T gm1inv, T F[4]) {
    T E = w.p * gm1inv + T(0.5) * w.r * (w.u * w.u + w.v * w.v);
    T m = w.r * w.v;
    F[0] = m;
    F[1] = m * w.u;
    F[2] = m * w.v + w.p;
    F[3] = w.v * (E + w.p);
}

// ---------------------------------------------------------------------------
// Variable policies.  PolAbs: the state holds the physical values (FP64 path).
// PolPert: the state holds perturbations about a uniform background W_bg and
// U(W_bg) (FP32 path); every conversion and flux below is the exact difference
// F(W_bg + W') - F(W_bg), so no large background value is ever rounded away.
// The increments of the acoustic operator and the Q2 evaluations are linear in
// the data and shift-invariant, so they act on perturbations unchanged.
// ---------------------------------------------------------------------------
template <class T>
struct PolAbs {
    T gamma, gm1inv;
    AF_HD T rho(T r) const { return r; }
    AF_HD T vu(T u) const { return u; }
    AF_HD T vv(T v) const { return v; }
    AF_HD T pr(T p) const { return p; }
    AF_HD Prim<T> centre(const T Ub[4], const Prim<T>& v00, const Prim<T>& v10, const Prim<T>& v01,
                         const Prim<T>& v11, const Prim<T>& eh0, const Prim<T>& eh1, const Prim<T>& ev0,
                         const Prim<T>& ev1) const {
        return recover_centre(Ub, v00, v10, v01, v11, eh0, eh1, ev0, ev1, gamma);
    }
    AF_HD void fx(const Prim<T>& w, T F[4]) const { flux_x(w, gm1inv, F); }
    AF_HD void fy(const Prim<T>& w, T F[4]) const { flux_y(w, gm1inv, F); }
};

template <class T>
struct PolPert {
    T gamma, gm1inv, r0, u0, v0, p0;
    T m0x, m0y, H0;    // background momentum and total enthalpy density E + p
    AF_HD T rho(T r) const { return r0 + r; }
    AF_HD T vu(T u) const { return u0 + u; }
    AF_HD T vv(T v) const { return v0 + v; }
    AF_HD T pr(T p) const { return p0 + p; }
    // E(W) - E(W_bg) from a perturbation
    AF_HD T energy(const Prim<T>& w) const {
        const T uu = u0 + w.u, vv = v0 + w.v;
        return w.p * gm1inv +
               T(0.5) * (w.r * (uu * uu + vv * vv) + r0 * (w.u * (T(2) * u0 + w.u) + w.v * (T(2) * v0 + w.v)));
    }
    AF_HD void cons(const Prim<T>& w, T U[4]) const {
        U[0] = w.r;
        U[1] = r0 * w.u + w.r * (u0 + w.u);
        U[2] = r0 * w.v + w.r * (v0 + w.v);
        U[3] = energy(w);
    }
    AF_HD Prim<T> centre(const T Ub[4], const Prim<T>& v00, const Prim<T>& v10, const Prim<T>& v01,
                         const Prim<T>& v11, const Prim<T>& eh0, const Prim<T>& eh1, const Prim<T>& ev0,
                         const Prim<T>& ev1) const {
        T Ua[4], U[4], sc[4], se[4];
        cons(v00, Ua);
        const Prim<T>* corners[3] = {&v10, &v01, &v11};
        const Prim<T>* edges[4] = {&eh0, &eh1, &ev0, &ev1};
#pragma unroll
        for (int k = 0; k < 4; ++k) { sc[k] = T(0); se[k] = T(0); }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cons(*corners[c], U);
#pragma unroll
            for (int k = 0; k < 4; ++k) sc[k] += U[k] - Ua[k];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            cons(*edges[c], U);
#pragma unroll
            for (int k = 0; k < 4; ++k) se[k] += U[k] - Ua[k];
        }
        T Uc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            Uc[k] = Ua[k] + T(2.25) * ((Ub[k] - Ua[k]) - sc[k] * T(1.0 / 36.0) - se[k] * T(1.0 / 9.0));
        Prim<T> w;
        w.r = Uc[0];
        const T ir = quot(T(1), r0 + Uc[0]);
        w.u = (Uc[1] - u0 * Uc[0]) * ir;
        w.v = (Uc[2] - v0 * Uc[0]) * ir;
        const T uu = u0 + w.u, vv = v0 + w.v;
        w.p = (gamma - T(1)) *
              (Uc[3] - T(0.5) * (w.r * (uu * uu + vv * vv) + r0 * (w.u * (T(2) * u0 + w.u) + w.v * (T(2) * v0 + w.v))));
        return w;
    }
    AF_HD void fx(const Prim<T>& w, T F[4]) const {
        const T uu = u0 + w.u, vv = v0 + w.v;
        const T m = r0 * w.u + w.r * uu;                 // rho u - rho0 u0
        const T Hp = energy(w) + w.p;                    // H - H0
        F[0] = m;
        F[1] = m0x * w.u + m * uu + w.p;
        F[2] = m0x * w.v + m * vv;
        F[3] = u0 * Hp + w.u * (H0 + Hp);
    }
    AF_HD void fy(const Prim<T>& w, T F[4]) const {
        const T uu = u0 + w.u, vv = v0 + w.v;
        const T m = r0 * w.v + w.r * vv;                 // rho v - rho0 v0
        const T Hp = energy(w) + w.p;
        F[0] = m;
        F[1] = m0y * w.u + m * uu;
        F[2] = m0y * w.v + m * vv + w.p;
        F[3] = v0 * Hp + w.v * (H0 + Hp);
    }
};

}  // namespace af
