// Algorithmic floating-point operation counts of one RB-TAI cell-update and of one
// cell's share of the reverse-mode (adjoint) step.
//
// Runs the library's own step arithmetic (af_kernels.h, the functions the kernels
// call) on the host with an operation-counting scalar, for the work that one cell
// owns: its recovered centre, the increments of its four nodes (V, Ev, Eh, C) for
// both durations, the point updates of its three targets (V, Ev, Eh) for both
// durations, their time-Simpson fluxes, one x- and one y-edge spatial Simpson flux
// and the average update.  Halo recomputation of a tiled kernel is not counted.
// The adjoint count (af_adjoint.h, the functions the adjoint kernels call) covers one
// cell's share of the reverse step: the forward intermediates recomputed from the
// time-n state (its centre and its four nodes' increments), the transposed fluxes and
// point updates of its three targets for both durations (each with the forward foot
// and Q2 evaluations it recomputes), the transposed increments of its four nodes (each
// re-forming its wedge sums) and its transposed centre recovery; every scattered
// contribution counts as one addition.  The kernels' additions of their LDS windows to
// global memory are not algorithmic work and are not counted.
// Every +, -, *, /, sqrt counts as one operation; a fused multiply-add counts as two.
//
// Build and run (host only):
//   hipcc -O1 -std=c++17 -I. -I../../include count_flops.cpp -o count_flops && ./count_flops
#include <cmath>
#include <cstdio>

static long g_add = 0, g_mul = 0, g_div = 0, g_sqrt = 0;

struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
    explicit operator int() const { return (int)v; }
};
inline Cnt operator+(Cnt a, Cnt b) { ++g_add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++g_add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++g_mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++g_div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
inline Cnt sqrt(Cnt a) { ++g_sqrt; return Cnt(std::sqrt(a.v)); }
inline Cnt rsqrt_of(Cnt a) { ++g_sqrt; ++g_div; return Cnt(1.0 / std::sqrt(a.v)); }   // a root and a quotient
inline Cnt quot(Cnt a, Cnt b) { return a / b; }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline Cnt floor(Cnt a) { return Cnt(std::floor(a.v)); }

#include "af_adjoint.h"
#include "af_kernels.h"

using namespace af;

// A smooth periodic 8x8 field (values only steer branches; counts do not depend on them).
struct HostAcc {
    Cnt s[16][8][8];
    Cnt C[4][8][8];
    Prim<Cnt> node(int fam, int i, int j) const {
        i = (i + 8) % 8;
        j = (j + 8) % 8;
        if (fam == F_C) return {C[0][j][i], C[1][j][i], C[2][j][i], C[3][j][i]};
        const int b = 4 + 4 * fam;
        return {s[b][j][i], s[b + 1][j][i], s[b + 2][j][i], s[b + 3][j][i]};
    }
};
struct HostInc {
    Cnt d[12][8][8];
    Cnt inc(int fam, int i, int j, int var) const { return d[fam * 3 + var][(j + 8) % 8][(i + 8) % 8]; }
};

static long total() { return g_add + g_mul + g_div + g_sqrt; }

// Adjoint accessors over a window of node-cells [-2, 6)^2 around cell (2, 2), with the
// window plane numbering of af_adjoint.h.
constexpr int kWX = 8;
struct HostStage {
    static constexpr int kRX = kWX, kPlane = kWX * kWX;
    Cnt a[40 * kWX * kWX];
    int base(int i, int j) const { return (j + 2) * kWX + (i + 2); }
    Cnt at(int pl, int b, int off) const { return a[b + pl * kPlane + off]; }
};
struct HostWin {
    static constexpr int kRX = kWX, kPlane = kWX * kWX;
    Cnt* a;
    int base(int i, int j) const { return (j + 2) * kWX + (i + 2); }
    void addb(int pl, int b, int off, Cnt v) const { a[b + pl * kPlane + off] = a[b + pl * kPlane + off] + v; }
    void node(int fam, int i, int j, const Cnt g[4]) const {
        const int b = fam == F_C ? 12 : 4 * fam, o = base(i, j);
        for (int q = 0; q < 4; ++q) addb(b + q, o, 0, g[q]);
    }
};
struct HostPlanes {   // cotangent planes by cell, periodic on the 8 x 8 field
    Cnt v[40][8][8];
    Cnt get(int k, int i, int j) const { return v[k][(j + 8) % 8][(i + 8) % 8]; }
};

int main() {
    static HostAcc A;
    static HostInc D;
    for (int j = 0; j < 8; ++j)
        for (int i = 0; i < 8; ++i) {
            double x = i / 8.0, y = j / 8.0;
            double W[4] = {1.0 + 0.01 * std::sin(6.283 * x), 0.3 + 0.01 * std::cos(6.283 * y), -0.2, 1.0};
            for (int f = 0; f < 3; ++f)
                for (int k = 0; k < 4; ++k) A.s[4 + 4 * f + k][j][i] = W[k];
            for (int k = 0; k < 4; ++k) A.C[k][j][i] = W[k];
            for (int k = 0; k < 4; ++k) A.s[k][j][i] = W[k];
            for (int k = 0; k < 12; ++k) D.d[k][j][i] = 1e-3;
        }
    const Cnt gamma = 1.4, lam0 = 0.1, lam1 = 0.2;
    unsigned st = 0;
    const PolAbs<Cnt> pol{gamma, Cnt(1.0 / 0.4)};
    long c0 = total();
    Cnt Ub[4] = {1.0, 0.3, -0.2, 2.6};
    recover_centre(Ub, A.node(F_V, 2, 2), A.node(F_V, 3, 2), A.node(F_V, 2, 3), A.node(F_V, 3, 3),
                   A.node(F_EH, 2, 2), A.node(F_EH, 2, 3), A.node(F_EV, 2, 2), A.node(F_EV, 3, 2), gamma);
    long centre = total() - c0;
    c0 = total();
    Cnt d[2][3];
    node_increments<F_V>(A, 2, 2, pol, lam0, lam1, d, st);
    long incV = total() - c0;
    c0 = total();
    node_increments<F_EV>(A, 2, 2, pol, lam0, lam1, d, st);
    node_increments<F_EH>(A, 2, 2, pol, lam0, lam1, d, st);
    long incE = total() - c0;
    c0 = total();
    node_increments<F_C>(A, 2, 2, pol, lam0, lam1, d, st);
    long incC = total() - c0;
    c0 = total();
    Prim<Cnt> w[3][2];
    w[0][0] = point_update<F_V, 0>(A, D, 2, 2, pol, lam0, st);
    w[0][1] = point_update<F_V, 0>(A, D, 2, 2, pol, lam1, st);
    w[1][0] = point_update<F_EV, 0>(A, D, 2, 2, pol, lam0, st);
    w[1][1] = point_update<F_EV, 0>(A, D, 2, 2, pol, lam1, st);
    w[2][0] = point_update<F_EH, 0>(A, D, 2, 2, pol, lam0, st);
    w[2][1] = point_update<F_EH, 0>(A, D, 2, 2, pol, lam1, st);
    long points = total() - c0;
    c0 = total();
    // time-Simpson fluxes of the owned targets: V (F and G), Ev (F), Eh (G)
    const Cnt gm1inv = Cnt(1.0) / (gamma - Cnt(1.0));
    auto tfl = [&](const Prim<Cnt>& a, const Prim<Cnt>& b, const Prim<Cnt>& c, bool xdir) {
        Cnt F0[4], Fh[4], F1[4];
        if (xdir) { flux_x(a, gm1inv, F0); flux_x(b, gm1inv, Fh); flux_x(c, gm1inv, F1); }
        else { flux_y(a, gm1inv, F0); flux_y(b, gm1inv, Fh); flux_y(c, gm1inv, F1); }
        for (int k = 0; k < 4; ++k) (void)((F0[k] + Cnt(4.0) * Fh[k] + F1[k]) * Cnt(1.0 / 6.0));
    };
    Prim<Cnt> w0 = A.node(F_V, 2, 2);
    tfl(w0, w[0][0], w[0][1], true);
    tfl(w0, w[0][0], w[0][1], false);
    tfl(A.node(F_EV, 2, 2), w[1][0], w[1][1], true);
    tfl(A.node(F_EH, 2, 2), w[2][0], w[2][1], false);
    long fluxes = total() - c0;
    c0 = total();
    // one x-edge and one y-edge spatial Simpson flux and the update, per component
    for (int k = 0; k < 4; ++k) {
        Cnt a = 1.0, b = 2.0, c = 3.0;
        Cnt Fl = (a + Cnt(4.0) * b + c) * Cnt(1.0 / 6.0);
        Cnt Gb = (a + Cnt(4.0) * b + c) * Cnt(1.0 / 6.0);
        Cnt Fr = Fl, Gt = Gb;
        (void)(Cnt(1.0) - lam1 * ((Fr - Fl) + (Gt - Gb)));
    }
    long update = total() - c0;
    long all = centre + incV + incE + incC + points + fluxes + update;
    const long f_add = g_add, f_mul = g_mul, f_div = g_div, f_sqrt = g_sqrt;

    // ---- adjoint: one cell's share of the reverse step ----
    static HostStage S;
    static Cnt winbuf[40 * kWX * kWX];
    static HostPlanes cot, lD;
    const HostWin O{winbuf};
    for (int pl = 0; pl < 40; ++pl)
        for (int y = 0; y < kWX; ++y)
            for (int x = 0; x < kWX; ++x) {
                const int i = x - 2, j = y - 2;
                Cnt v = 1e-3;
                if (pl < 12) v = A.s[4 + pl][(j + 8) % 8][(i + 8) % 8];
                else if (pl < 16) v = A.C[pl - 12][(j + 8) % 8][(i + 8) % 8];
                S.a[pl * kWX * kWX + y * kWX + x] = v;
            }
    for (int k = 0; k < 40; ++k)
        for (int j = 0; j < 8; ++j)
            for (int i = 0; i < 8; ++i) { cot.v[k][j][i] = 1e-2; lD.v[k][j][i] = 1e-2; }
    const long a0 = total();
    // forward intermediates (centre of the cell, increments of its four nodes)
    recover_centre(Ub, A.node(F_V, 2, 2), A.node(F_V, 3, 2), A.node(F_V, 2, 3), A.node(F_V, 3, 3),
                   A.node(F_EH, 2, 2), A.node(F_EH, 2, 3), A.node(F_EV, 2, 2), A.node(F_EV, 3, 2), gamma);
    node_increments<F_V>(A, 2, 2, pol, lam0, lam1, d, st);
    node_increments<F_EV>(A, 2, 2, pol, lam0, lam1, d, st);
    node_increments<F_EH>(A, 2, 2, pol, lam0, lam1, d, st);
    node_increments<F_C>(A, 2, 2, pol, lam0, lam1, d, st);
    const long adj_fwd = total() - a0;
    long a1 = total();
    unsigned fix = point_adj_target<F_V, 0, 0>(S, cot, O, 2, 2, gamma, lam0, lam1);
    fix |= point_adj_target<F_EV, 0, 0>(S, cot, O, 2, 2, gamma, lam0, lam1);
    fix |= point_adj_target<F_EH, 0, 0>(S, cot, O, 2, 2, gamma, lam0, lam1);
    if (fix) std::fprintf(stderr, "warning: a counted target's Picard stages left one cell\n");
    const long adj_points = total() - a1;
    a1 = total();
    incr_adj<F_V>(A, lD, O, 2, 2, gamma, lam0, lam1);
    incr_adj<F_EV>(A, lD, O, 2, 2, gamma, lam0, lam1);
    incr_adj<F_EH>(A, lD, O, 2, 2, gamma, lam0, lam1);
    incr_adj<F_C>(A, lD, O, 2, 2, gamma, lam0, lam1);
    const long adj_incr = total() - a1;
    a1 = total();
    const Cnt lW[4] = {1e-2, 1e-2, 1e-2, 1e-2};
    centre_adj(A, O, 2, 2, lW, gamma);
    const long adj_centre = total() - a1;
    const long adj_all = adj_fwd + adj_points + adj_incr + adj_centre;
    std::fprintf(stderr, "adjoint: forward intermediates %ld, points %ld, increments %ld, centre %ld\n", adj_fwd,
                 adj_points, adj_incr, adj_centre);
    std::printf("{\"centre\": %ld, \"increments_V\": %ld, \"increments_Ev_Eh\": %ld, \"increments_C\": %ld, "
                "\"point_updates\": %ld, \"target_fluxes\": %ld, \"edge_fluxes_update\": %ld, "
                "\"adds\": %ld, \"muls\": %ld, \"divs\": %ld, \"sqrts\": %ld, "
                "\"flops_per_cell_update\": %ld, \"adjoint_forward_intermediates\": %ld, \"adjoint_points\": %ld, "
                "\"adjoint_increments\": %ld, \"adjoint_centre\": %ld, \"adjoint_flops_per_cell\": %ld}\n",
                centre, incV, incE, incC, points, fluxes, update, f_add, f_mul, f_div, f_sqrt, all, adj_fwd, adj_points,
                adj_incr, adj_centre, adj_all);
    return 0;
}
