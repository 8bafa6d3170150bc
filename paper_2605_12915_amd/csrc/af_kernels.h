// Node-level pieces of the RB-TAI step expressed against an accessor, shared by
// the multi-kernel path and the fused LDS-tiled kernel.
//
// An accessor A provides
//   Prim<T> A.node(fam, ci, cj)       primitive value of node family fam of cell
//                                     (ci, cj) (fam = F_C: the recovered centre),
// and an increment accessor D provides
//   T D.inc(fam, ci, cj, var)         acoustic increment (var 0: du, 1: dv, 2: dp)
//                                     of the node for the tau being processed.
// Cell indices are relative to whatever origin the accessor uses.
#pragma once
#include "af_device.h"

namespace af {

// Nine nodes of cell (ci, cj) in [x-node][y-node] order (Sec. 2; Sec. 4 R_Delta).
template <class T, class A>
AF_HD void cell_nodes(const A& acc, int ci, int cj, Prim<T> n[3][3]) {
    n[0][0] = acc.node(F_V, ci, cj);      n[1][0] = acc.node(F_EH, ci, cj);     n[2][0] = acc.node(F_V, ci + 1, cj);
    n[0][1] = acc.node(F_EV, ci, cj);     n[1][1] = acc.node(F_C, ci, cj);      n[2][1] = acc.node(F_EV, ci + 1, cj);
    n[0][2] = acc.node(F_V, ci, cj + 1);  n[1][2] = acc.node(F_EH, ci, cj + 1); n[2][2] = acc.node(F_V, ci + 1, cj + 1);
}

template <class T, class A>
AF_HD void cell_puv(const A& acc, int ci, int cj, T f[3][3][3]) {
    Prim<T> n[3][3];
    cell_nodes<T>(acc, ci, cj, n);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            f[0][a][b] = n[a][b].p;
            f[1][a][b] = n[a][b].u;
            f[2][a][b] = n[a][b].v;
        }
}

// Accumulate every wedge of node family FAM at (i, j) (Sec. 3.1: four quadrants at
// a vertex, two half-planes at an edge midpoint, the full disk at a centre).
template <int FAM, class T, class A>
AF_HD void node_wedges(const A& acc, int i, int j, NodeAcc<T>& na) {
    T f[3][3][3];
    if constexpr (FAM == F_V) {
        cell_puv<T>(acc, i, j, f);         wedge_acc<W_V_NE, 0, 0>(f, na);
        cell_puv<T>(acc, i - 1, j, f);     wedge_acc<W_V_NW, 1, 0>(f, na);
        cell_puv<T>(acc, i - 1, j - 1, f); wedge_acc<W_V_SW, 1, 1>(f, na);
        cell_puv<T>(acc, i, j - 1, f);     wedge_acc<W_V_SE, 0, 1>(f, na);
    } else if constexpr (FAM == F_EV) {
        cell_puv<T>(acc, i, j, f);         wedge_acc<W_EV_R, 0, 2>(f, na);
        cell_puv<T>(acc, i - 1, j, f);     wedge_acc<W_EV_L, 1, 2>(f, na);
    } else if constexpr (FAM == F_EH) {
        cell_puv<T>(acc, i, j, f);         wedge_acc<W_EH_U, 2, 0>(f, na);
        cell_puv<T>(acc, i, j - 1, f);     wedge_acc<W_EH_D, 2, 1>(f, na);
    } else {
        cell_puv<T>(acc, i, j, f);         wedge_acc<W_C, 2, 2>(f, na);
    }
}

// Node freezing (Sec. 6.1 step 1) and the increments for two durations
// tau_k = lam_k h (k = 0: dt/2, 1: dt).  Sets SB_CFL if c_K dt / h > 1/2 and
// SB_NONPHYS if the node state is not physical.
template <int FAM, class T, class A, class Pol>
AF_HD void node_increments(const A& acc, int i, int j, const Pol& pol, T lam0, T lam1, T inc[2][3],
                           unsigned& st) {
    const Prim<T> Wn = acc.node(FAM, i, j);
    const T rK = pol.rho(Wn.r), pK = pol.pr(Wn.p);
    if (!(rK > T(0)) || !(pK > T(0))) st |= SB_NONPHYS;
    // c = sqrt(gamma p / rho) and Z = rho c from one reciprocal square root:
    // 1 / Z = (gamma p rho)^(-1/2), c = gamma p / Z, Z = gamma p rho / Z
    const T gp = pol.gamma * pK, q = gp * rK;
    const T iZ = rsqrt_of(q);
    const T c = gp * iZ, Z = q * iZ;
    NodeAcc<T> na;
    na.zero();
    node_wedges<FAM>(acc, i, j, na);
    T r0 = c * lam0, r1 = c * lam1;
    if (!(r1 <= T(0.5))) st |= SB_CFL;
    node_increment(na, r0, Z, iZ, inc[0]);
    node_increment(na, r1, Z, iZ, inc[1]);
}

template <int FAM>
struct FamOffset;
template <> struct FamOffset<F_V> { static constexpr double ox = 0.0, oy = 0.0; };
template <> struct FamOffset<F_EV> { static constexpr double ox = 0.0, oy = 0.5; };
template <> struct FamOffset<F_EH> { static constexpr double ox = 0.5, oy = 0.0; };

// The same offsets for a target family known only at run time (cell units).
template <class T>
AF_HD T fam_ox(int fam) { return fam == F_EH ? T(0.5) : T(0); }
template <class T>
AF_HD T fam_oy(int fam) { return fam == F_EV ? T(0.5) : T(0); }

// Locate an offset (cell units, relative to the target's own cell) in its cell:
// integer shift and local coordinate in [-1, 1].  A displacement of one cell or
// more (or NaN) raises SB_FOOT and is replaced by the node itself, which keeps
// every gather inside the two-cell halo.
template <class T>
AF_HD void locate(T off, T o, int& cell, T& xi, unsigned& st) {
    if (!(fabs(off - o) < T(1))) { st |= SB_FOOT; off = o; }
    T fl = floor(off);
    cell = (int)fl;
    xi = T(2) * (off - fl) - T(1);
}

// Transported (SCHEME 0, eq. transported-update) or additive (SCHEME 1,
// eq. barsukow-additive) point update of the target of family fam (F_V, F_EV or
// F_EH) at (i, j) for duration tau = lam h (Sec. 6.1 steps 3-4).  The family may be
// a run-time value (lanes of one wavefront then share one instruction stream) or a
// constant (point_update<FAM, ...>).
// The convective foot of the target of family fam at (i, j) (node value WP) after
// tau = lam h, by the two Picard stages (eq. adv-footpoint; Sec. 6.1 step 3): the
// foot's cell (ci, cj) and its local coordinates (xi, eta) in [-1, 1].
template <class T, class A, class Pol>
AF_HD void picard_foot(const A& acc, int fam, int i, int j, const Pol& pol, T lam, const Prim<T>& WP, int& ci,
                       int& cj, T& xi, T& eta, unsigned& st) {
    const T ox = fam_ox<T>(fam), oy = fam_oy<T>(fam);
    int cx, cy;
    T xm, xp, ym, yp;
    // first Picard step: at a node the reconstruction equals the node value
    locate(ox - lam * pol.vu(WP.u), ox, cx, xi, st);
    locate(oy - lam * pol.vv(WP.v), oy, cy, eta, st);
    lag_pm(xi, xm, xp);
    lag_pm(eta, ym, yp);
    T fu[3][3], fv[3][3];
    {
        Prim<T> n[3][3];
        cell_nodes<T>(acc, i + cx, j + cy, n);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) { fu[a][b] = n[a][b].u; fv[a][b] = n[a][b].v; }
    }
    T u1 = q2(xm, xp, ym, yp, fu), v1 = q2(xm, xp, ym, yp, fv);
    // second Picard step from P with the velocity at the first foot
    locate(ox - lam * pol.vu(u1), ox, cx, xi, st);
    locate(oy - lam * pol.vv(v1), oy, cy, eta, st);
    ci = i + cx;
    cj = j + cy;
}

template <int SCHEME, class T, class A, class D, class Pol>
AF_HD Prim<T> point_update_f(const A& acc, const D& dinc, int fam, int i, int j, const Pol& pol, T lam,
                             unsigned& st) {
    Prim<T> WP = acc.node(fam, i, j);
    int ci, cj;
    T xi, eta, xm, xp, ym, yp;
    picard_foot(acc, fam, i, j, pol, lam, WP, ci, cj, xi, eta, st);
    lag_pm(xi, xm, xp);
    lag_pm(eta, ym, yp);
    T fr[3][3], fu[3][3], fv[3][3], fp[3][3];
    {
        Prim<T> n[3][3];
        cell_nodes<T>(acc, ci, cj, n);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                fr[a][b] = n[a][b].r; fu[a][b] = n[a][b].u; fv[a][b] = n[a][b].v; fp[a][b] = n[a][b].p;
            }
    }
    Prim<T> Wf{q2(xm, xp, ym, yp, fr), q2(xm, xp, ym, yp, fu), q2(xm, xp, ym, yp, fv), q2(xm, xp, ym, yp, fp)};
    T du, dv, dp, rho_over_c2;
    if constexpr (SCHEME == 0) {
        T g[3][3];
#pragma unroll
        for (int var = 0; var < 3; ++var) {
            g[0][0] = dinc.inc(F_V, ci, cj, var);      g[1][0] = dinc.inc(F_EH, ci, cj, var);
            g[2][0] = dinc.inc(F_V, ci + 1, cj, var);  g[0][1] = dinc.inc(F_EV, ci, cj, var);
            g[1][1] = dinc.inc(F_C, ci, cj, var);      g[2][1] = dinc.inc(F_EV, ci + 1, cj, var);
            g[0][2] = dinc.inc(F_V, ci, cj + 1, var);  g[1][2] = dinc.inc(F_EH, ci, cj + 1, var);
            g[2][2] = dinc.inc(F_V, ci + 1, cj + 1, var);
            T val = q2(xm, xp, ym, yp, g);
            if (var == 0) du = val; else if (var == 1) dv = val; else dp = val;
        }
        rho_over_c2 = quot(pol.rho(Wf.r), pol.gamma * pol.pr(Wf.p));    // 1 / c^2 at the foot
    } else {
        du = dinc.inc(fam, i, j, 0);
        dv = dinc.inc(fam, i, j, 1);
        dp = dinc.inc(fam, i, j, 2);
        rho_over_c2 = quot(pol.rho(WP.r), pol.gamma * pol.pr(WP.p));    // frozen 1 / c^2 at P
    }
    return Prim<T>{Wf.r + dp * rho_over_c2, Wf.u + du, Wf.v + dv, Wf.p + dp};
}

template <int FAM, int SCHEME, class T, class A, class D, class Pol>
AF_HD Prim<T> point_update(const A& acc, const D& dinc, int i, int j, const Pol& pol, T lam, unsigned& st) {
    return point_update_f<SCHEME>(acc, dinc, FAM, i, j, pol, lam, st);
}

// Both durations of one target at once.  The two Picard stages of both durations
// normally stay in one cell, fixed by the sign of the node velocity; that cell's
// nine nodes and both increment sets are gathered once and every stage is checked
// to stay in it.  Lanes whose feet leave it take the general path above, which
// performs the same arithmetic (so the results do not depend on the path).
template <int SCHEME, class T, class A, class D, class Pol>
AF_HD void point_update_pair_f(const A& acc, const D& d0, const D& d1, int fam, int i, int j, const Pol& pol,
                               T lam0, T lam1, unsigned& st, Prim<T>& wh, Prim<T>& w1) {
    const T ox = fam_ox<T>(fam), oy = fam_oy<T>(fam);
    const Prim<T> WP = acc.node(fam, i, j);
    // candidate cell from the longer first-stage displacement
    const T uP = pol.vu(WP.u), vP = pol.vv(WP.v);
    const T ex = ox - lam1 * uP, ey = oy - lam1 * vP;
    bool fast = (fabs(ex - ox) < T(1)) && (fabs(ey - oy) < T(1));
    int cx = 0, cy = 0;
    Prim<T> wr[2];
    if (fast) {
        const T fcx = floor(ex), fcy = floor(ey);
        cx = (int)fcx;
        cy = (int)fcy;
        const int ci = i + cx, cj = j + cy;
        T fr[3][3], fu[3][3], fv[3][3], fp[3][3];
        {
            Prim<T> n[3][3];
            cell_nodes<T>(acc, ci, cj, n);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    fr[a][b] = n[a][b].r; fu[a][b] = n[a][b].u; fv[a][b] = n[a][b].v; fp[a][b] = n[a][b].p;
                }
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const T lam = t ? lam1 : lam0;
            T xi, eta, xm, xp, ym, yp, fl;
            // first Picard stage
            T o1x = ox - lam * uP, o1y = oy - lam * vP;
            fl = floor(o1x); fast = fast && (fl == fcx); xi = T(2) * (o1x - fl) - T(1);
            fl = floor(o1y); fast = fast && (fl == fcy); eta = T(2) * (o1y - fl) - T(1);
            lag_pm(xi, xm, xp);
            lag_pm(eta, ym, yp);
            const T u1 = q2(xm, xp, ym, yp, fu), v1 = q2(xm, xp, ym, yp, fv);
            // second stage
            T o2x = ox - lam * pol.vu(u1), o2y = oy - lam * pol.vv(v1);
            fast = fast && (fabs(o2x - ox) < T(1)) && (fabs(o2y - oy) < T(1));
            fl = floor(o2x); fast = fast && (fl == fcx); xi = T(2) * (o2x - fl) - T(1);
            fl = floor(o2y); fast = fast && (fl == fcy); eta = T(2) * (o2y - fl) - T(1);
            lag_pm(xi, xm, xp);
            lag_pm(eta, ym, yp);
            Prim<T> Wf{q2(xm, xp, ym, yp, fr), q2(xm, xp, ym, yp, fu), q2(xm, xp, ym, yp, fv), q2(xm, xp, ym, yp, fp)};
            T du, dv, dp, rho_over_c2;
            if constexpr (SCHEME == 0) {
                // increments of the candidate cell's nine nodes for this duration,
                // gathered per duration to bound the live set
                const D& dd = t ? d1 : d0;
                T g[3][3][3];
#pragma unroll
                for (int var = 0; var < 3; ++var) {
                    g[var][0][0] = dd.inc(F_V, ci, cj, var);      g[var][1][0] = dd.inc(F_EH, ci, cj, var);
                    g[var][2][0] = dd.inc(F_V, ci + 1, cj, var);  g[var][0][1] = dd.inc(F_EV, ci, cj, var);
                    g[var][1][1] = dd.inc(F_C, ci, cj, var);      g[var][2][1] = dd.inc(F_EV, ci + 1, cj, var);
                    g[var][0][2] = dd.inc(F_V, ci, cj + 1, var);  g[var][1][2] = dd.inc(F_EH, ci, cj + 1, var);
                    g[var][2][2] = dd.inc(F_V, ci + 1, cj + 1, var);
                }
                du = q2(xm, xp, ym, yp, g[0]);
                dv = q2(xm, xp, ym, yp, g[1]);
                dp = q2(xm, xp, ym, yp, g[2]);
                rho_over_c2 = quot(pol.rho(Wf.r), pol.gamma * pol.pr(Wf.p));
            } else {
                const D& dd = t ? d1 : d0;
                du = dd.inc(fam, i, j, 0);
                dv = dd.inc(fam, i, j, 1);
                dp = dd.inc(fam, i, j, 2);
                rho_over_c2 = quot(pol.rho(WP.r), pol.gamma * pol.pr(WP.p));
            }
            wr[t] = Prim<T>{Wf.r + dp * rho_over_c2, Wf.u + du, Wf.v + dv, Wf.p + dp};
        }
    }
    if (fast) {
        wh = wr[0];
        w1 = wr[1];
    } else {
        wh = point_update_f<SCHEME>(acc, d0, fam, i, j, pol, lam0, st);
        w1 = point_update_f<SCHEME>(acc, d1, fam, i, j, pol, lam1, st);
    }
}

template <int FAM, int SCHEME, class T, class A, class D, class Pol>
AF_HD void point_update_pair(const A& acc, const D& d0, const D& d1, int i, int j, const Pol& pol, T lam0, T lam1,
                             unsigned& st, Prim<T>& wh, Prim<T>& w1) {
    point_update_pair_f<SCHEME>(acc, d0, d1, FAM, i, j, pol, lam0, lam1, st, wh, w1);
}

}  // namespace af
