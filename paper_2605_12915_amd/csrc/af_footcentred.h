// Foot-centred exact frozen-acoustic point update (App. C; Sec. 4, the paragraph on an
// exact frozen acoustic update), FP64, for the multi-kernel path (af_f64.hip); host and
// device code, so that a host build can check it against the oracle (tests/fc_host.cpp).
//
// For a target P and a duration tau: the convective foot F by the two Picard stages of
// the transported update (eq. adv-footpoint), the frozen state W* = W_h^n(F) of the
// cellwise Q2 reconstruction, c* = sqrt(gamma p* / rho*), Z* = rho* c*, and the disk
// of radius R = c* tau / h (cell units) about F, which must stay inside the half-cell
// footprint |F - P| + R < 1/2 in each direction (eq. fc-half-footprint).  With pi = p / Z*
// the exact solution of the frozen acoustic system at F after tau is written with
// spherical means M_r[f] = (1 / 2 pi) int_{|z| < 1} f(F + r z) (1 - |z|^2)^(-1/2) dz of
// the continuous piecewise-Q2 data:
//   pi(F) = M_R[pi_0] + R M_R[z . grad pi_0] - R M_R[g],        g = div u_0,
//   u(F)  = u_0(F) - R M_R[grad pi_0] + int_0^R r M_r[grad g] dr.
// The last integral (grad g distributional: g jumps across grid lines) equals, after
// exchanging the integration order and integrating by parts over the disk's pieces,
// (R / 2 pi) int_0^{2 pi} e_theta int_0^{pi/2} g(F + R sin(psi) e_theta) dpsi dtheta:
// one more sum over the nodes of M_R.  Density from the transported update's linear
// closure rho* + (p - p*) / c*^2.
//
// Quadrature: polar coordinates about F with |z| = sin(psi) (absorbing the weight), the
// angle split at multiples of pi/4, where a grid line touches the circle (with cuts
// graded towards the tangency) and where a ray passes through a grid corner, and each
// ray's psi range split where it crosses a grid line, so that every piece lies in one
// cell; 32 Gauss points per angular piece, clustered towards both ends by
// theta = t0 + (t1 - t0)(1 - cos(pi s)) / 2 (square-root behaviour at a tangency), and
// 10 per radial piece.  The footprint keeps the disk inside the 2 x 2 cells around P,
// so at most one vertical and one horizontal grid line cut it.
#pragma once
#include <hip/hip_runtime.h>

#include "af_gauss.h"
#include "af_internal.h"
#include "af_kernels.h"

namespace af {

constexpr double kFcPi = 3.14159265358979323846;

// Nodal values of one cell, minus the frozen values: p, u, v at [a][b] (a along x).
struct FcCell { double p[3][3], u[3][3], v[3][3]; };

// Quadrature sums over the disk: M_R of (p - p*), z . grad p, g, grad p; history
// (1 / 2 pi) int int g e_theta dpsi dtheta.
struct FcSums { double m0, m1, mg, mx, my, hx, hy; };

AF_HD void fc_lagrange(double s, double L[3], double dL[3]) {
    // Lagrange basis at s = -1, 0, 1 and its derivative in cell units (d/dX = 2 d/ds)
    L[0] = 0.5 * s * (s - 1.0);
    L[1] = 1.0 - s * s;
    L[2] = 0.5 * s * (s + 1.0);
    dL[0] = 2.0 * s - 1.0;
    dL[1] = -4.0 * s;
    dL[2] = 2.0 * s + 1.0;
}

// Add one quadrature point (local coordinates s, t in the cell; unit-disk position z;
// weights w of M_R and wh of the history term).
AF_HD void fc_point(const FcCell& c, double s, double t, double zx, double zy, double ct,
                                         double st, double w, double wh, FcSums& S) {
    double Lx[3], dLx[3], Ly[3], dLy[3];
    fc_lagrange(s, Lx, dLx);
    fc_lagrange(t, Ly, dLy);
    double p0 = 0.0, px = 0.0, py = 0.0, ux = 0.0, vy = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double r = Lx[0] * c.p[0][b] + Lx[1] * c.p[1][b] + Lx[2] * c.p[2][b];
        const double rd = dLx[0] * c.p[0][b] + dLx[1] * c.p[1][b] + dLx[2] * c.p[2][b];
        const double ud = dLx[0] * c.u[0][b] + dLx[1] * c.u[1][b] + dLx[2] * c.u[2][b];
        p0 += Ly[b] * r;
        px += Ly[b] * rd;
        py += dLy[b] * r;
        ux += Ly[b] * ud;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) vy += Lx[a] * (dLy[0] * c.v[a][0] + dLy[1] * c.v[a][1] + dLy[2] * c.v[a][2]);
    const double g = ux + vy;
    S.m0 += w * p0;
    S.m1 += w * (zx * px + zy * py);
    S.mg += w * g;
    S.mx += w * px;
    S.my += w * py;
    S.hx += wh * g * ct;
    S.hy += wh * g * st;
}

// Sort a short array in place (insertion sort).
AF_HD void fc_sort(double* a, int n) {
    for (int k = 1; k < n; ++k) {
        const double v = a[k];
        int m = k - 1;
        while (m >= 0 && a[m] > v) { a[m + 1] = a[m]; --m; }
        a[m + 1] = v;
    }
}

// The disk sums for the foot at (Xf, Yf) relative to the target's cell (i, j) (cell
// units) and radius R, 0 < R, |Xf - ox| + R < 1/2, |Yf - oy| + R < 1/2.  ws: frozen
// state, subtracted from the nodal values (uniform data give zero sums exactly).
template <class A>
AF_HD void fc_disk(const A& acc, int i, int j, double Xf, double Yf, double R, const Prim<double>& ws,
                        FcSums& S) {
    S = FcSums{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // the grid lines that cut the disk: at most one in each direction
    const int kx = (int)floor(Xf + R), ky = (int)floor(Yf + R);
    const bool hx = (double)kx > Xf - R && (double)kx < Xf + R;
    const bool hy = (double)ky > Yf - R && (double)ky < Yf + R;
    const double lam = hx ? ((double)kx - Xf) / R : 0.0, mu = hy ? ((double)ky - Yf) / R : 0.0;
    double cuts[32];
    int nc = 0;
    for (int q = 0; q < 8; ++q) cuts[nc++] = q * (0.25 * kFcPi);
    auto tangency = [&](double l, double base) {
        const double a = acos(fmin(1.0, fabs(l)));
        cuts[nc++] = base - a;
        cuts[nc++] = base + a;
        const double gr[3] = {0.25, 1.0, 4.0};
        for (int q = 0; q < 3; ++q) {
            const double d = gr[q] * fabs(l);
            if (d < a) {
                cuts[nc++] = base - a + d;
                cuts[nc++] = base + a - d;
            }
        }
    };
    if (hx) tangency(lam, lam > 0.0 ? 0.0 : kFcPi);
    if (hy) tangency(mu, mu > 0.0 ? 0.5 * kFcPi : 1.5 * kFcPi);
    if (hx && hy) {
        const double dx = (double)kx - Xf, dy = (double)ky - Yf;
        if (dx * dx + dy * dy < R * R) cuts[nc++] = atan2(dy, dx);
    }
    for (int q = 0; q < nc; ++q) {
        double c = fmod(cuts[q], 2.0 * kFcPi);
        if (c < 0.0) c += 2.0 * kFcPi;
        cuts[q] = c;
    }
    cuts[nc++] = 2.0 * kFcPi;
    fc_sort(cuts, nc);
    const double inv2pi = 1.0 / (2.0 * kFcPi);
    for (int q = 0; q + 1 < nc; ++q) {
        const double t0 = cuts[q], t1 = cuts[q + 1];
        if (t1 - t0 < 1e-15) continue;
        // lines crossed by the rays of this piece, in the order of increasing radius
        // (the same for every ray of the piece)
        const double tm = 0.5 * (t0 + t1), cm = cos(tm), sm = sin(tm);
        int nx_ = 0;
        int axis[2];
        double qm[2];
        if (hx && lam / cm > 0.0 && lam / cm < 1.0) { axis[nx_] = 0; qm[nx_] = lam / cm; ++nx_; }
        if (hy && mu / sm > 0.0 && mu / sm < 1.0) { axis[nx_] = 1; qm[nx_] = mu / sm; ++nx_; }
        if (nx_ == 2 && qm[1] < qm[0]) {
            const int a = axis[0]; axis[0] = axis[1]; axis[1] = a;
            const double b = qm[0]; qm[0] = qm[1]; qm[1] = b;
        }
        for (int seg = 0; seg <= nx_; ++seg) {
            // this radial piece's cell, from its middle on the middle ray
            const double p0m = seg == 0 ? 0.0 : asin(qm[seg - 1]);
            const double p1m = seg == nx_ ? 0.5 * kFcPi : asin(qm[seg]);
            const double rm = sin(0.5 * (p0m + p1m));
            const int cx = (int)floor(Xf + R * rm * cm), cy = (int)floor(Yf + R * rm * sm);
            FcCell C;
            {
                Prim<double> n[3][3];
                cell_nodes<double>(acc, i + cx, j + cy, n);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        C.p[a][b] = n[a][b].p - ws.p;
                        C.u[a][b] = n[a][b].u - ws.u;
                        C.v[a][b] = n[a][b].v - ws.v;
                    }
            }
#pragma unroll 1
            for (int k = 0; k < 32; ++k) {
                const double th = t0 + 0.5 * (t1 - t0) * (1.0 - kGaussCos32[k]);
                const double wth = kGaussW32[k] * 0.5 * (t1 - t0) * kFcPi * kGaussSin32[k];
                const double ct = cos(th), st = sin(th);
                auto psi_at = [&](int c) -> double {
                    const double qv = axis[c] == 0 ? lam / ct : mu / st;
                    return asin(fmin(1.0, fmax(0.0, qv)));
                };
                const double p0 = seg == 0 ? 0.0 : psi_at(seg - 1);
                const double p1 = seg == nx_ ? 0.5 * kFcPi : psi_at(seg);
                const bool whole = nx_ == 0;   // psi over [0, pi/2]: tabulated sines
#pragma unroll 2
                for (int m = 0; m < 10; ++m) {
                    const double wps = (p1 - p0) * kGaussW10[m];
                    const double rho = whole ? kGaussSinHalf10[m] : sin(p0 + (p1 - p0) * kGaussX10[m]);
                    const double zx = rho * ct, zy = rho * st;
                    const double X = Xf + R * zx, Y = Yf + R * zy;
                    fc_point(C, 2.0 * (X - cx) - 1.0, 2.0 * (Y - cy) - 1.0, zx, zy, ct, st,
                             wth * wps * rho * inv2pi, wth * wps * inv2pi, S);
                }
            }
        }
    }
}

// New point value of the target of family fam at (i, j) after tau = lam h.
template <class A>
AF_HD Prim<double> fc_point_update(const A& acc, int fam, int i, int j, double gamma, double lam,
                                        unsigned& st) {
    const PolAbs<double> pol{gamma, 1.0 / (gamma - 1.0)};
    const Prim<double> WP = acc.node(fam, i, j);
    int ci, cj;
    double xi, eta, xm, xp, ym, yp;
    picard_foot(acc, fam, i, j, pol, lam, WP, ci, cj, xi, eta, st);
    lag_pm(xi, xm, xp);
    lag_pm(eta, ym, yp);
    double fr[3][3], fu[3][3], fv[3][3], fp[3][3];
    {
        Prim<double> n[3][3];
        cell_nodes<double>(acc, ci, cj, n);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                fr[a][b] = n[a][b].r; fu[a][b] = n[a][b].u; fv[a][b] = n[a][b].v; fp[a][b] = n[a][b].p;
            }
    }
    const Prim<double> ws{q2(xm, xp, ym, yp, fr), q2(xm, xp, ym, yp, fu), q2(xm, xp, ym, yp, fv),
                          q2(xm, xp, ym, yp, fp)};
    if (!(ws.r > 0.0) || !(ws.p > 0.0)) {
        st |= SB_NONPHYS;
        return ws;
    }
    const double c2 = gamma * ws.p / ws.r, c = sqrt(c2), Z = ws.r * c, R = c * lam;
    // foot relative to the target's cell, and its displacement from the target
    const double Xf = (double)(ci - i) + 0.5 * (xi + 1.0), Yf = (double)(cj - j) + 0.5 * (eta + 1.0);
    const double dx = Xf - fam_ox<double>(fam), dy = Yf - fam_oy<double>(fam);
    if (!(fabs(dx) + R < 0.5) || !(fabs(dy) + R < 0.5)) {
        st |= SB_FOOTPRINT;
        return ws;
    }
    if (!(R > 0.0)) return ws;
    FcSums S;
    fc_disk(acc, i, j, Xf, Yf, R, ws, S);
    const double p = ws.p + S.m0 + R * S.m1 - Z * R * S.mg;
    const double u = ws.u - (R / Z) * S.mx + R * S.hx;
    const double v = ws.v - (R / Z) * S.my + R * S.hy;
    return Prim<double>{ws.r + (p - ws.p) / c2, u, v, p};
}

}  // namespace af
