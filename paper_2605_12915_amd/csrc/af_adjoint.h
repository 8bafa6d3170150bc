// Arithmetic of the reverse-mode step (transposed Sec. 6.1 dataflow), written once
// for the scalar type T and against small accessor types, so that the adjoint
// kernels (af_adjoint.hip, T = double, LDS windows) and the host operation count
// (count_flops.cpp, an operation-counting scalar) run the very same code.
//
// Accessors:
//   S  staged forward state: S.base(i, j), S.at(plane, base, off) with the window
//      plane numbering (0..11 point values fam * 4 + (rho, u, v, p), 12..15 recovered
//      centres, 16..39 increments tau * 12 + fam * 3 + (u, v, p)); row stride S_::kRX.
//   O  scatter target with the same plane numbering (its own row stride O_::kRX):
//      O.base(i, j), O.addb(plane, base, off, value), O.node(fam, i, j, g[4]); every
//      add is one accumulation.
//   A  forward nodes by cell: A.node(fam, i, j) (fam = F_C: recovered centre).
//   CT cotangent of the step's output: CT.get(plane, i, j) (periodic).
//   LD cotangent of the increments: LD.get(tau * 12 + fam * 3 + q, i, j).
// The floor() that locates a foot is piecewise constant: its derivative is zero.
#pragma once
#include "af_kernels.h"

namespace af {

// Family of node [a][b] of a cell, and its first plane in the scatter window (point
// values fam * 4, centre 12).
AF_HD constexpr int fam_of(int a, int b) {
    return (a == 1 && b == 1) ? F_C : (a == 1 ? F_EH : (b == 1 ? F_EV : F_V));
}
AF_HD constexpr int win_plane(int fam) { return fam == F_C ? 12 : 4 * fam; }

template <class T>
AF_HD void lagr(T s, T l[3], T dl[3]) {
    l[0] = T(0.5) * s * (s - T(1));
    l[1] = T(1) - s * s;
    l[2] = T(0.5) * s * (s + T(1));
    dl[0] = s - T(0.5);
    dl[1] = T(-2) * s;
    dl[2] = s + T(0.5);
}

// Flux Jacobians transposed: g += (dF/dW)^T nu, W = (rho, u, v, p).
// (Each product shared by several terms is formed once, as the compiled code does; the
// one quotient, 1 / (gamma - 1), is the same in every call and formed once per thread.)
template <class T>
AF_HD void flux_x_T(const Prim<T>& w, T gamma, const T nu[4], T g[4]) {
    const T gm1i = T(1) / (gamma - T(1));
    const T uu = w.u * w.u, uv = w.u * w.v, ru = w.r * w.u;
    const T q2 = T(0.5) * (uu + w.v * w.v);
    const T E = w.p * gm1i + w.r * q2;
    g[0] += nu[0] * w.u + nu[1] * uu + nu[2] * uv + nu[3] * w.u * q2;
    g[1] += nu[0] * w.r + nu[1] * T(2) * ru + nu[2] * w.r * w.v + nu[3] * (E + w.p + ru * w.u);
    g[2] += nu[2] * ru + nu[3] * ru * w.v;
    g[3] += nu[1] + nu[3] * w.u * gamma * gm1i;
}

template <class T>
AF_HD void flux_y_T(const Prim<T>& w, T gamma, const T nu[4], T g[4]) {
    const T gm1i = T(1) / (gamma - T(1));
    const T vv = w.v * w.v, uv = w.u * w.v, rv = w.r * w.v;
    const T q2 = T(0.5) * (w.u * w.u + vv);
    const T E = w.p * gm1i + w.r * q2;
    g[0] += nu[0] * w.v + nu[1] * uv + nu[2] * vv + nu[3] * w.v * q2;
    g[1] += nu[1] * rv + nu[3] * rv * w.u;
    g[2] += nu[0] * w.r + nu[1] * w.r * w.u + nu[2] * T(2) * rv + nu[3] * (E + w.p + rv * w.v);
    g[3] += nu[2] + nu[3] * w.v * gamma * gm1i;
}

// Transposed point update of target FAM at (i, j) for the duration tau = lam h;
// WP = the target's time-n value.  SCHEME 0: transported update (the increments are
// interpolated at the foot, the density closure uses c^2 at the foot); SCHEME 1:
// additive update (the target's own increments, c^2 frozen at the target).
// The forward value w is recomputed here and its cotangent formed from the flux
// cotangents: lw = ws * (dF/dW)^T nuF + ws * (dG/dW)^T nuG (+ extra: the cotangent
// of the new point value itself, for the full step).  The contributions to the
// target's own node (through the first foot position) are added to gself, those to
// the nodes of the two foot cells go to the window, one base offset per cell.
//
// The two Picard stages normally lie in one foot cell; then each node's contribution
// through the first stage's u1 = Q2(u) is added to its second-stage contribution
// before a single scatter.  MODE 0 does that and returns true for a target whose
// stages lie in different cells, whose first-stage contributions it leaves out; MODE 1
// recomputes such a target and scatters only those (the caller runs it for the rare
// wavefronts that need it, so the common path keeps one scatter per node and plane).
template <int FAM, int SCHEME, int MODE, class T, class S_, class O_>
AF_HD bool point_update_adj(const S_& S, const O_& O, int t, int i, int j, const Prim<T>& WP, T gamma, T lam,
                            const T nuF[4], const T nuG[4], T ws, const T* extra, T gself[4]) {
    const T ox = T(FamOffset<FAM>::ox), oy = T(FamOffset<FAM>::oy);
    constexpr int RX = O_::kRX, SRX = S_::kRX;   // row strides of the window and of the staged state
    unsigned st = 0;
    // ---- forward recomputation ----
    int cx1, cy1, cx2, cy2;
    T xi1, eta1, xi2, eta2;
    locate(ox - lam * WP.u, ox, cx1, xi1, st);
    locate(oy - lam * WP.v, oy, cy1, eta1, st);
    T lx1[3], dlx1[3], ly1[3], dly1[3];
    lagr(xi1, lx1, dlx1);
    lagr(eta1, ly1, dly1);
    T u1 = T(0), v1 = T(0), du1x = T(0), du1y = T(0), dv1x = T(0), dv1y = T(0);
    T w1[3][3];   // tensor weights of the first foot (reused by the reverse scatter)
    const int wb1 = O.base(i + cx1, j + cy1), sb1 = S.base(i + cx1, j + cy1);
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int f = fam_of(a, b), soff = (b == 2 ? SRX : 0) + (a == 2 ? 1 : 0);
                const T nu_ = S.at(win_plane(f) + 1, sb1, soff), nv_ = S.at(win_plane(f) + 2, sb1, soff);
                const T w = lx1[a] * ly1[b], wx = dlx1[a] * ly1[b], wy = lx1[a] * dly1[b];
                w1[a][b] = w;
                u1 += w * nu_;
                v1 += w * nv_;
                du1x += wx * nu_;
                du1y += wy * nu_;
                dv1x += wx * nv_;
                dv1y += wy * nv_;
            }
    }
    locate(ox - lam * u1, ox, cx2, xi2, st);
    locate(oy - lam * v1, oy, cy2, eta2, st);
    T lx2[3], dlx2[3], ly2[3], dly2[3];
    lagr(xi2, lx2, dlx2);
    lagr(eta2, ly2, dly2);
    const int ci = i + cx2, cj = j + cy2;
    T Wf[4] = {T(0), T(0), T(0), T(0)}, dWx[4] = {T(0), T(0), T(0), T(0)}, dWy[4] = {T(0), T(0), T(0), T(0)};
    T Df[3] = {T(0), T(0), T(0)}, dDx[3] = {T(0), T(0), T(0)}, dDy[3] = {T(0), T(0), T(0)};
    T w2[3][3];   // tensor weights of the second foot (reused by the reverse scatter)
    const int wb2 = O.base(ci, cj), sb2 = S.base(ci, cj);
    {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T w = lx2[a] * ly2[b], wx = dlx2[a] * ly2[b], wy = lx2[a] * dly2[b];
                w2[a][b] = w;
                const int f = fam_of(a, b), soff = (b == 2 ? SRX : 0) + (a == 2 ? 1 : 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T v = S.at(win_plane(f) + q, sb2, soff);
                    Wf[q] += w * v; dWx[q] += wx * v; dWy[q] += wy * v;
                }
                if constexpr (SCHEME == 0) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const T v = S.at(16 + t * 12 + f * 3 + q, sb2, soff);
                        Df[q] += w * v; dDx[q] += wx * v; dDy[q] += wy * v;
                    }
                }
            }
    }
    const int wbP = O.base(i, j);
    if constexpr (SCHEME == 1) {
        const int sbP = S.base(i, j);
#pragma unroll
        for (int q = 0; q < 3; ++q) Df[q] = S.at(16 + t * 12 + FAM * 3 + q, sbP, 0);
    }
    // ---- reverse ----
    // compose: rho = rho_f + dp rho_K / (gamma p_K), u = u_f + du, v = v_f + dv, p = p_f + dp,
    // with K the foot (SCHEME 0) or the target (SCHEME 1)
    const T rK = SCHEME == 0 ? Wf[0] : WP.r, pK = SCHEME == 0 ? Wf[3] : WP.p;
    const T qinv = T(1) / (gamma * pK), rq = rK * qinv;
    T lw[4] = {T(0), T(0), T(0), T(0)};
    {
        const Prim<T> w{Wf[0] + Df[2] * rq, Wf[1] + Df[0], Wf[2] + Df[1], Wf[3] + Df[2]};
        T nu[4];
        if constexpr (FAM != F_EH) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = ws * nuF[k];
            flux_x_T(w, gamma, nu, lw);
        }
        if constexpr (FAM != F_EV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = ws * nuG[k];
            flux_y_T(w, gamma, nu, lw);
        }
        if (extra)
#pragma unroll
            for (int k = 0; k < 4; ++k) lw[k] += extra[k];
    }
    T lWf[4], lDf[3];
    lDf[0] = lw[1];
    lDf[1] = lw[2];
    lDf[2] = lw[3] + lw[0] * rq;
    lWf[1] = lw[1];
    lWf[2] = lw[2];
    const T ldq = lw[0] * Df[2] * qinv;
    if constexpr (SCHEME == 0) {
        lWf[0] = lw[0] + ldq;
        lWf[3] = lw[3] - ldq * gamma * rq;   // rho_K / p_K = gamma rq
    } else {
        lWf[0] = lw[0];
        lWf[3] = lw[3];
        // the frozen rho_K / (gamma p_K) at the target, and its own increments
        gself[0] += ldq;
        gself[3] -= ldq * gamma * rq;
#pragma unroll
        for (int q = 0; q < 3; ++q) O.addb(16 + t * 12 + FAM * 3 + q, wbP, 0, lDf[q]);
    }
    // foot position: xi2 = 2 (off - floor(off)) - 1, off = ox - lam u1
    T lxi2 = T(0), leta2 = T(0);
#pragma unroll
    for (int q = 0; q < 4; ++q) { lxi2 += lWf[q] * dWx[q]; leta2 += lWf[q] * dWy[q]; }
    if constexpr (SCHEME == 0)
#pragma unroll
        for (int q = 0; q < 3; ++q) { lxi2 += lDf[q] * dDx[q]; leta2 += lDf[q] * dDy[q]; }
    const T lu1 = T(-2) * lam * lxi2, lv1 = T(-2) * lam * leta2;
    // Q2 values at the foot -> nodes of the foot cell, and the first stage's
    // u1 = Q2(u) at (xi1, eta1): lu1, lv1 -> u, v of the first foot cell's nodes.  When
    // both stages lie in one cell (the usual case) each node's two contributions are
    // added before one scatter.
    const bool same = wb1 == wb2;
    if constexpr (MODE == 1) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const T v = w1[a][b];
                const int f = fam_of(a, b), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
                O.addb(win_plane(f) + 1, wb1, off, v * lu1);
                O.addb(win_plane(f) + 2, wb1, off, v * lv1);
            }
        return false;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const T w = w2[a][b], v = w1[a][b];
            const int f = fam_of(a, b), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
            O.addb(win_plane(f), wb2, off, w * lWf[0]);
            O.addb(win_plane(f) + 1, wb2, off, w * lWf[1] + (same ? v * lu1 : T(0)));
            O.addb(win_plane(f) + 2, wb2, off, w * lWf[2] + (same ? v * lv1 : T(0)));
            O.addb(win_plane(f) + 3, wb2, off, w * lWf[3]);
            if constexpr (SCHEME == 0)
#pragma unroll
                for (int q = 0; q < 3; ++q) O.addb(16 + t * 12 + f * 3 + q, wb2, off, w * lDf[q]);
        }
    const T lxi1 = lu1 * du1x + lv1 * dv1x, leta1 = lu1 * du1y + lv1 * dv1y;
    gself[1] += T(-2) * lam * lxi1;
    gself[2] += T(-2) * lam * leta1;
    return !same;
}

// Reverse sweep of one target (family FAM of node-cell (i, j)): the adjoints of the
// edge fluxes it feeds, from the averages' cotangents, then of its three time levels
// (w^n directly, w^{n+1/2} and w^{n+1} through the transposed point update).
// MODE 0 returns a bit per duration (1: tau = dt/2, 2: tau = dt) whose Picard stages
// left one cell; MODE 1, given those bits, scatters the first-stage contributions that
// MODE 0 left out (everything it needs is reloaded, so that the common path does not
// keep it live).
template <int FAM, int SCHEME, int MODE, class T, class S_, class CT, class O_>
AF_HD unsigned point_adj_target(const S_& S, const CT& cot1, const O_& O, int i, int j, T gamma, T lam0, T lam1,
                                unsigned fix = 0) {
    // cotangents of the time-integrated edge fluxes at this node: F at V and Ev, G at
    // V and Eh; spatial Simpson weights 1/6 (V, two edges each) and 4/6 (edge midpoints)
    T nuF[4] = {T(0), T(0), T(0), T(0)}, nuG[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T lij = cot1.get(k, i, j);
        const T muF_ij = lam1 * (lij - cot1.get(k, i - 1, j));
        const T muG_ij = lam1 * (lij - cot1.get(k, i, j - 1));
        if constexpr (FAM == F_V) {
            const T lijm = cot1.get(k, i, j - 1), limj = cot1.get(k, i - 1, j), limjm = cot1.get(k, i - 1, j - 1);
            const T muF_ijm = lam1 * (lijm - limjm);
            const T muG_imj = lam1 * (limj - limjm);
            nuF[k] = (muF_ij + muF_ijm) * T(1.0 / 6.0);
            nuG[k] = (muG_ij + muG_imj) * T(1.0 / 6.0);
        } else if constexpr (FAM == F_EV) {
            nuF[k] = muF_ij * T(4.0 / 6.0);
        } else {
            nuG[k] = muG_ij * T(4.0 / 6.0);
        }
    }
    const int wb = O.base(i, j), sb = S.base(i, j);
    const int pl = win_plane(FAM);
    const Prim<T> w0{S.at(pl, sb, 0), S.at(pl + 1, sb, 0), S.at(pl + 2, sb, 0), S.at(pl + 3, sb, 0)};
    T g[4] = {T(0), T(0), T(0), T(0)};
    if constexpr (MODE == 1) {
        if (fix & 1u)
            point_update_adj<FAM, SCHEME, 1>(S, O, 0, i, j, w0, gamma, lam0, nuF, nuG, T(4.0 / 6.0), (const T*)nullptr, g);
        if (fix & 2u) {
            const T extra[4] = {cot1.get(4 + 4 * FAM, i, j), cot1.get(5 + 4 * FAM, i, j), cot1.get(6 + 4 * FAM, i, j),
                                cot1.get(7 + 4 * FAM, i, j)};
            point_update_adj<FAM, SCHEME, 1>(S, O, 1, i, j, w0, gamma, lam1, nuF, nuG, T(1.0 / 6.0), extra, g);
        }
        return 0u;
    }
    // time level n (time-Simpson weight 1/6): the node itself
    {
        T nu[4];
        if constexpr (FAM != F_EH) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = nuF[k] * T(1.0 / 6.0);
            flux_x_T(w0, gamma, nu, g);
        }
        if constexpr (FAM != F_EV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) nu[k] = nuG[k] * T(1.0 / 6.0);
            flux_y_T(w0, gamma, nu, g);
        }
    }
    // n + 1/2 (weight 4/6) and n + 1 (weight 1/6; also an output of the step)
    unsigned out = 0u;
    if (point_update_adj<FAM, SCHEME, 0>(S, O, 0, i, j, w0, gamma, lam0, nuF, nuG, T(4.0 / 6.0), (const T*)nullptr,
                                         g))
        out |= 1u;
    const T extra[4] = {cot1.get(4 + 4 * FAM, i, j), cot1.get(5 + 4 * FAM, i, j), cot1.get(6 + 4 * FAM, i, j),
                        cot1.get(7 + 4 * FAM, i, j)};
    if (point_update_adj<FAM, SCHEME, 0>(S, O, 1, i, j, w0, gamma, lam1, nuF, nuG, T(1.0 / 6.0), extra, g))
        out |= 2u;
#pragma unroll
    for (int q = 0; q < 4; ++q) O.addb(pl + q, wb, 0, g[q]);
    return out;
}

// Transposed 1-D Lagrange-to-monomial transform (see mono1): (lc0, lc1, lc2) -> (lf0, lf1, lf2).
template <int XC, class T>
AF_HD void mono1_T(T c0, T c1, T c2, T& f0, T& f1, T& f2) {
    if constexpr (XC == 0) { f0 = c0 - T(3) * c1 + T(2) * c2; f1 = T(4) * c1 - T(4) * c2; f2 = -c1 + T(2) * c2; }
    else if constexpr (XC == 1) { f0 = c1 + T(2) * c2; f1 = T(-4) * c1 - T(4) * c2; f2 = c0 + T(3) * c1 + T(2) * c2; }
    else { f0 = -c1 + T(2) * c2; f1 = c0 - T(4) * c2; f2 = c1 + T(2) * c2; }
}

// Transposed wedge: adjoint of the accumulators -> adjoint of the cell's nodal (p, u, v),
// scattered to the nodes of cell (ci, cj).
template <int W, int XC, int YC, class T, class O_>
AF_HD void wedge_adj(const T la[6][4], const O_& O, int ci, int cj) {
    constexpr int RX = O_::kRX;
    T lc[3][3][3];
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) lc[v][a][b] = T(0);
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) {
            if (al + be == 0) continue;
            const int m = al + be - 1;
            const double* B = kBlk[W][al][be];
            T sp = T(0), su = T(0), sv = T(0);
            if (B[0] != 0.0) sp += T(B[0]) * la[0][m];
            if (B[3] != 0.0) sp += T(B[3]) * la[2][m];
            if (B[6] != 0.0) sp += T(B[6]) * la[4][m];
            if (B[1] != 0.0) su += T(B[1]) * la[1][m];
            if (B[4] != 0.0) su += T(B[4]) * la[3][m];
            if (B[7] != 0.0) su += T(B[7]) * la[5][m];
            if (B[2] != 0.0) sv += T(B[2]) * la[1][m];
            if (B[5] != 0.0) sv += T(B[5]) * la[3][m];
            if (B[8] != 0.0) sv += T(B[8]) * la[5][m];
            lc[0][al][be] = sp;
            lc[1][al][be] = su;
            lc[2][al][be] = sv;
        }
    T lf[3][3][3];   // [var][x-node][y-node]
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        T lg[3][3];  // [alpha][y-node]
#pragma unroll
        for (int al = 0; al < 3; ++al) mono1_T<YC>(lc[v][al][0], lc[v][al][1], lc[v][al][2], lg[al][0], lg[al][1], lg[al][2]);
#pragma unroll
        for (int b = 0; b < 3; ++b) mono1_T<XC>(lg[0][b], lg[1][b], lg[2][b], lf[v][0][b], lf[v][1][b], lf[v][2][b]);
    }
    const int wb = O.base(ci, cj);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int pl = win_plane(fam_of(a, b)), off = (b == 2 ? RX : 0) + (a == 2 ? 1 : 0);
            O.addb(pl + 1, wb, off, lf[1][a][b]);
            O.addb(pl + 2, wb, off, lf[2][a][b]);
            O.addb(pl + 3, wb, off, lf[0][a][b]);
        }
}

// Transposed node increments of node FAM at (i, j): Horner in r, freezing c_K and Z_K,
// transposed monomial blocks and Lagrange-to-monomial transforms of every wedge.  A node
// whose six increment cotangents are all zero contributes nothing and is skipped.
template <int FAM, class T, class A_, class LD_, class O_>
AF_HD void incr_adj(const A_& A, const LD_& LD, const O_& O, int i, int j, T gamma, T lam0, T lam1) {
    T li[2][3];
    bool any = false;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            li[t][q] = LD.get(t * 12 + FAM * 3 + q, i, j);
            any = any || (li[t][q] != T(0));
        }
    if (!any) return;
    const Prim<T> W = A.node(FAM, i, j);
    // as in the forward freezing: 1 / Z = (gamma p rho)^(-1/2), c = gamma p / Z, Z = rho c
    const T gp = gamma * W.p, q = gp * W.r;
    const T iZ = rsqrt_of(q);
    const T c = gp * iZ, Z = q * iZ;
    NodeAcc<T> na;
    na.zero();
    node_wedges<FAM>(A, i, j, na);
    T la[6][4];
#pragma unroll
    for (int ch = 0; ch < 6; ++ch)
#pragma unroll
        for (int m = 0; m < 4; ++m) la[ch][m] = T(0);
    T lc = T(0), lZ = T(0), liZ = T(0);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const T lam = t ? lam1 : lam0;
        const T r = c * lam;
        T s[6], ds[6];
#pragma unroll
        for (int ch = 0; ch < 6; ++ch) {
            s[ch] = ((na.a[ch][3] * r + na.a[ch][2]) * r + na.a[ch][1]) * r + na.a[ch][0];
            ds[ch] = (T(3) * na.a[ch][3] * r + T(2) * na.a[ch][2]) * r + na.a[ch][1];
        }
        // inc0 = r (s2 iZ + s3), inc1 = r (s4 iZ + s5), inc2 = r (s0 + Z s1)
        const T l0r = li[t][0] * r, l1r = li[t][1] * r, l2r = li[t][2] * r;
        T ls[6];
        ls[2] = l0r * iZ;
        ls[3] = l0r;
        ls[4] = l1r * iZ;
        ls[5] = l1r;
        ls[0] = l2r;
        ls[1] = l2r * Z;
        T rp = T(1);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int ch = 0; ch < 6; ++ch) la[ch][m] += ls[ch] * rp;
            rp = rp * r;
        }
        const T lr = li[t][0] * (s[2] * iZ + s[3] + r * (ds[2] * iZ + ds[3])) +
                     li[t][1] * (s[4] * iZ + s[5] + r * (ds[4] * iZ + ds[5])) +
                     li[t][2] * (s[0] + Z * s[1] + r * (ds[0] + Z * ds[1]));
        lc += lam * lr;
        liZ += l0r * s[2] + l1r * s[4];
        lZ += l2r * s[1];
    }
    lZ += -iZ * iZ * liZ;
    // c = sqrt(gamma p / rho), Z = rho c: dc/drho = -c / (2 rho) = -c^2 / (2 Z),
    // dc/dp = c / (2 p) = gamma / (2 Z), dZ/drho = c / 2, dZ/dp = Z / (2 p) = gamma rho / (2 Z)
    {
        const int wb = O.base(i, j);
        const T hiZ = T(0.5) * iZ;
        O.addb(win_plane(FAM), wb, 0, lc * (-c * c * hiZ) + lZ * (T(0.5) * c));
        O.addb(win_plane(FAM) + 3, wb, 0, lc * (gamma * hiZ) + lZ * (gamma * W.r * hiZ));
    }
    if constexpr (FAM == F_V) {
        wedge_adj<W_V_NE, 0, 0>(la, O, i, j);
        wedge_adj<W_V_NW, 1, 0>(la, O, i - 1, j);
        wedge_adj<W_V_SW, 1, 1>(la, O, i - 1, j - 1);
        wedge_adj<W_V_SE, 0, 1>(la, O, i, j - 1);
    } else if constexpr (FAM == F_EV) {
        wedge_adj<W_EV_R, 0, 2>(la, O, i, j);
        wedge_adj<W_EV_L, 1, 2>(la, O, i - 1, j);
    } else if constexpr (FAM == F_EH) {
        wedge_adj<W_EH_U, 2, 0>(la, O, i, j);
        wedge_adj<W_EH_D, 2, 1>(la, O, i, j - 1);
    } else {
        wedge_adj<W_C, 2, 2>(la, O, i, j);
    }
}

template <class T>
AF_HD void cons_T(const Prim<T>& w, T gamma, const T lU[4], T g[4]) {
    // U = (rho, rho u, rho v, p/(gamma-1) + rho (u^2+v^2)/2)
    const T q2 = T(0.5) * (w.u * w.u + w.v * w.v);
    g[0] = lU[0] + w.u * lU[1] + w.v * lU[2] + q2 * lU[3];
    g[1] = w.r * lU[1] + w.r * w.u * lU[3];
    g[2] = w.r * lU[2] + w.r * w.v * lU[3];
    g[3] = lU[3] / (gamma - T(1));
}

// Transposed centre recovery of cell (i, j) for the centre cotangent lW: the averages'
// cotangent (plane 16 + k of the window, weight 9/4) and the point values of the cell's
// eight boundary nodes (through U(W) at corners, weight -1/16, and edge midpoints, -1/4).
template <class T, class A_, class O_>
AF_HD void centre_adj(const A_& A, const O_& O, int i, int j, const T lW[4], T gamma) {
    const Prim<T> Wc = A.node(F_C, i, j);
    // W = prim(U_c): rho = U0, u = U1/U0, v = U2/U0, p = (g-1)(U3 - (U1 u + U2 v)/2)
    const T ir = T(1) / Wc.r, gm1 = gamma - T(1);
    T lU[4];
    lU[0] = lW[0] - lW[1] * Wc.u * ir - lW[2] * Wc.v * ir + lW[3] * gm1 * T(0.5) * (Wc.u * Wc.u + Wc.v * Wc.v);
    lU[1] = lW[1] * ir - lW[3] * gm1 * Wc.u;
    lU[2] = lW[2] * ir - lW[3] * gm1 * Wc.v;
    lU[3] = lW[3] * gm1;
    // U_c = 9/4 [Ubar - sum_corners U / 36 - sum_edges U / 9]
    const int wb = O.base(i, j);
#pragma unroll
    for (int k = 0; k < 4; ++k) O.addb(16 + k, wb, 0, T(2.25) * lU[k]);
    T lc[4], le[4], g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) { lc[k] = -lU[k] * T(1.0 / 16.0); le[k] = -lU[k] * T(0.25); }
    cons_T(A.node(F_V, i, j), gamma, lc, g);          O.node(F_V, i, j, g);
    cons_T(A.node(F_V, i + 1, j), gamma, lc, g);      O.node(F_V, i + 1, j, g);
    cons_T(A.node(F_V, i, j + 1), gamma, lc, g);      O.node(F_V, i, j + 1, g);
    cons_T(A.node(F_V, i + 1, j + 1), gamma, lc, g);  O.node(F_V, i + 1, j + 1, g);
    cons_T(A.node(F_EH, i, j), gamma, le, g);         O.node(F_EH, i, j, g);
    cons_T(A.node(F_EH, i, j + 1), gamma, le, g);     O.node(F_EH, i, j + 1, g);
    cons_T(A.node(F_EV, i, j), gamma, le, g);         O.node(F_EV, i, j, g);
    cons_T(A.node(F_EV, i + 1, j), gamma, le, g);     O.node(F_EV, i + 1, j, g);
}

}  // namespace af
