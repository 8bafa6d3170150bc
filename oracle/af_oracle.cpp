// Plain FP64 CPU oracle of the fully discrete RB-TAI Active Flux step.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference
// that the GPU library is checked against.  It is called only by the test suite,
// by the package smoke check and by the benchmark's CPU-baseline leg; the product
// path never links or calls it.  It shares no code, header, table or constant
// with the GPU library: every quantity below is recomputed here from the paper's
// definitions (Duraisamy, "Fully Discrete Active Flux Method based on Transported
// Acoustic Increments for the Compressible Euler Equations").
//
// Structure follows the algorithm of Sec. 6.1 step by step:
//   1. centre recovery from the conservative Simpson constraint (Sec. 2,
//      eq. center-node; Sec. 4, the U^C_{ij} formula),
//   2. node freezing rho_K, c_K, Z_K at V, Ev, Eh and recovered C nodes (Sec. 6.1
//      step 1, Sec. 3.1),
//   3. exact node-centred acoustic operator: four quadrants at a vertex, two
//      half-planes at an edge midpoint, the full disk at a centre (Sec. 3.1,
//      Sec. 4 "Cellwise Q2 reconstruction"), evaluated with the compact monomial
//      block of App. D (eq. compact-monomial-block),
//   4. cellwise Q2 interpolants of the increments (Sec. 4, R_Delta; Sec. 6.1 step 2),
//   5. two-Picard convective foot from the time-n reconstruction (eq. adv-footpoint,
//      Sec. 6.1 step 3) and the transported point update with the density tied to
//      the pressure increment through the frozen invariant (Sec. 6.1 step 4),
//   6. space-time Simpson fluxes and the one-stage conservative average update
//      (Sec. 3, eq. af-average-update; Sec. 6.1).
// Optionally (scheme = 1) the additive RB point update of eq. barsukow-additive.
//
// Every function is templated on the scalar so that the same code runs in
// double and in std::complex<double> (complex-step directional derivatives:
// Im f(x + i e v) / e); branches and floor() act on the real part only.
//
// Readings of the paper taken here (silent or garbled passages):
//  * App. B / App. D orientation: cell nodal arrays are indexed [x-node][y-node].
//  * Foot location: the displacement is formed in cell units relative to the
//    target's own cell and the containing cell chosen by floor(); R_h and I_h are
//    continuous across faces, so the choice on a face is immaterial.
//  * Entropy functional -int rho log(p / rho^gamma) dA: tensor Simpson rule over the
//    nine Q2 nodes of every cell.
//  * Acoustic CFL guard: c_K tau / h <= 1/2 at every node for tau = dt; the foot
//    displacement must stay below one cell.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cplx& x) { return x.real(); }

inline int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

// ---------------------------------------------------------------------------
// App. D geometric quantities
// ---------------------------------------------------------------------------
// mu_{mn}^Theta = int_Theta cos^m(t) sin^n(t) dt for a wedge made of whole quadrants
// (quadrant k covers [k pi/2, (k+1) pi/2]).  On the first quadrant the integral is
// B((m+1)/2, (n+1)/2) / 2; the other quadrants follow by t -> pi - t, pi + t, 2pi - t.
double mu_quadrant(int k, int m, int n) {
    double base = 0.5 * std::tgamma(0.5 * (m + 1)) * std::tgamma(0.5 * (n + 1)) /
                  std::tgamma(0.5 * (m + n + 2));
    bool cneg = (k == 1 || k == 2), sneg = (k == 2 || k == 3);
    double s = 1.0;
    if (cneg && (m & 1)) s = -s;
    if (sneg && (n & 1)) s = -s;
    return s * base;
}

double mu_wedge(int quad_mask, int m, int n) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k)
        if (quad_mask & (1 << k)) s += mu_quadrant(k, m, n);
    return s;
}

// zeta_j = sqrt(pi) Gamma((j+1)/2) / Gamma(j/2 + 1)
double zeta(int j) { return std::sqrt(M_PI) * std::tgamma(0.5 * (j + 1)) / std::tgamma(0.5 * j + 1.0); }

// The 3x3 block C_ab^Theta of eq. compact-monomial-block; input and output ordered
// (pi, u, v).  Row-major into C[9].
void monomial_block(int a, int b, int quad_mask, double C[9]) {
    int q = a + b;
    double chi = (q == 0) ? 1.0 : 1.0 + 1.0 / q;
    double g = q + 1 + 3.0 * chi;
    double M = mu_wedge(quad_mask, a, b) * zeta(q + 1);
    double X = mu_wedge(quad_mask, a + 2, b) * zeta(q + 3);
    double Y = mu_wedge(quad_mask, a + 1, b + 1) * zeta(q + 3);
    double Z = mu_wedge(quad_mask, a, b + 2) * zeta(q + 3);
    double Px = (q + 2) * mu_wedge(quad_mask, a + 1, b) * zeta(q + 2);
    double Py = (q + 2) * mu_wedge(quad_mask, a, b + 1) * zeta(q + 2);
    double k = 1.0 / (4.0 * M_PI);
    C[0] = k * (q + 1) * M;  C[1] = -k * Px;                 C[2] = -k * Py;
    C[3] = -k * Px;          C[4] = k * (g * X - chi * M);   C[5] = k * g * Y;
    C[6] = -k * Py;          C[7] = k * g * Y;               C[8] = k * (g * Z - chi * M);
    if (q == 0) {
        int nq = 0;
        for (int kq = 0; kq < 4; ++kq) nq += (quad_mask >> kq) & 1;
        double omega = nq * 0.25;                 // |Theta| / 2pi
        C[4] += 2.0 * omega / 3.0;
        C[8] += 2.0 * omega / 3.0;
    }
}

struct BlockTable {
    // blk[mask][a][b][9] for every wedge mask used by the node types
    double blk[16][3][3][9];
    BlockTable() {
        std::memset(blk, 0, sizeof(blk));
        for (int mask = 1; mask < 16; ++mask)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) monomial_block(a, b, mask, blk[mask][a][b]);
    }
};
const BlockTable& blocks() { static BlockTable t; return t; }

// Node families and their wedges (Sec. 3.1 and Sec. 6.1 step 1):
// a vertex sees four quadrants, an edge midpoint two half-planes, a centre the disk.
enum NodeType { NV = 0, NEV = 1, NEH = 2, NC = 3 };
struct WedgeDef { int dci, dcj, mask; };     // owning cell offset from the node's (i,j)
struct NodeDef { double ox, oy; int nw; WedgeDef w[4]; };
const NodeDef kNodes[4] = {
    // V_ij at (x_i, y_j): NE -> C_ij, NW -> C_{i-1,j}, SW -> C_{i-1,j-1}, SE -> C_{i,j-1}
    {0.0, 0.0, 4, {{0, 0, 1}, {-1, 0, 2}, {-1, -1, 4}, {0, -1, 8}}},
    // Ev_ij at (x_i, y_{j+1/2}): right half [-pi/2, pi/2] -> C_ij, left -> C_{i-1,j}
    {0.0, 0.5, 2, {{0, 0, 8 | 1}, {-1, 0, 2 | 4}, {0, 0, 0}, {0, 0, 0}}},
    // Eh_ij at (x_{i+1/2}, y_j): upper half [0, pi] -> C_ij, lower -> C_{i,j-1}
    {0.5, 0.0, 2, {{0, 0, 1 | 2}, {0, -1, 4 | 8}, {0, 0, 0}, {0, 0, 0}}},
    // C_ij at the cell centre: full disk -> C_ij
    {0.5, 0.5, 1, {{0, 0, 15}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}}},
};

// Coefficients of the 1-D Lagrange basis on the nodes X0, X0+1/2, X0+1 as
// polynomials in X: L[a][k] = coefficient of X^k in L_a(X).
void lagrange_monomials(double X0, double L[3][3]) {
    double xs[3] = {X0, X0 + 0.5, X0 + 1.0};
    for (int a = 0; a < 3; ++a) {
        int b = (a + 1) % 3, c = (a + 2) % 3;
        double den = (xs[a] - xs[b]) * (xs[a] - xs[c]);
        // (X - xb)(X - xc) = X^2 - (xb + xc) X + xb xc
        L[a][0] = xs[b] * xs[c] / den;
        L[a][1] = -(xs[b] + xs[c]) / den;
        L[a][2] = 1.0 / den;
    }
}

// Exact frozen acoustic operator of one wedge applied to one cell's Q2 data.
// f[var][ax][by]: nodal values of (pi, u, v) on the cell's 3x3 node lattice,
// [x-node][y-node]; (X0, Y0): position of the cell's lower-left node relative to
// the node K, in units of h.  Returns the (pi, u, v) contribution at radius r.
template <class T>
void wedge_apply(int mask, double X0, double Y0, const T f[3][3][3], T r, T out[3]) {
    double Lx[3][3], Ly[3][3];
    lagrange_monomials(X0, Lx);
    lagrange_monomials(Y0, Ly);
    T coef[3][3][3];       // [var][alpha][beta]
    for (int v = 0; v < 3; ++v)
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be) {
                T s = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) s += f[v][a][b] * (Lx[a][al] * Ly[b][be]);
                coef[v][al][be] = s;
            }
    const BlockTable& bt = blocks();
    out[0] = out[1] = out[2] = 0.0;
    for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) {
            const double* C = bt.blk[mask][al][be];
            T rp = 1.0;
            for (int k = 0; k < al + be; ++k) rp *= r;
            for (int o = 0; o < 3; ++o) {
                T s = C[3 * o + 0] * coef[0][al][be] + C[3 * o + 1] * coef[1][al][be] +
                      C[3 * o + 2] * coef[2][al][be];
                out[o] += rp * s;
            }
        }
}

// ---------------------------------------------------------------------------
// Grid state
// ---------------------------------------------------------------------------
template <class T>
struct Prim { T r, u, v, p; };

template <class T>
struct Grid {
    int nx, ny;
    double h, gamma;
    const T* s;                   // 16 planes (ny, nx)
    std::vector<Prim<T>> C;       // recovered centres
    int64_t N() const { return (int64_t)nx * ny; }
    T at(int plane, int i, int j) const { return s[(int64_t)plane * N() + (int64_t)wrap(j, ny) * nx + wrap(i, nx)]; }
    Prim<T> node(int fam, int i, int j) const {
        if (fam == NC) return C[(int64_t)wrap(j, ny) * nx + wrap(i, nx)];
        int b = 4 + 4 * fam;
        return {at(b, i, j), at(b + 1, i, j), at(b + 2, i, j), at(b + 3, i, j)};
    }
    // The nine primitive Q2 nodes of cell (ci, cj), [x-node][y-node].
    void cell_nodes(int ci, int cj, Prim<T> n[3][3]) const {
        n[0][0] = node(NV, ci, cj);     n[1][0] = node(NEH, ci, cj);     n[2][0] = node(NV, ci + 1, cj);
        n[0][1] = node(NEV, ci, cj);    n[1][1] = node(NC, ci, cj);      n[2][1] = node(NEV, ci + 1, cj);
        n[0][2] = node(NV, ci, cj + 1); n[1][2] = node(NEH, ci, cj + 1); n[2][2] = node(NV, ci + 1, cj + 1);
    }
};

template <class T>
void cons_of(const Prim<T>& w, double g, T U[4]) {
    U[0] = w.r;
    U[1] = w.r * w.u;
    U[2] = w.r * w.v;
    U[3] = w.p / (g - 1.0) + 0.5 * w.r * (w.u * w.u + w.v * w.v);
}

template <class T>
Prim<T> prim_of(const T U[4], double g) {
    Prim<T> w;
    w.r = U[0];
    w.u = U[1] / U[0];
    w.v = U[2] / U[0];
    w.p = (g - 1.0) * (U[3] - 0.5 * (U[1] * U[1] + U[2] * U[2]) / U[0]);
    return w;
}

// Step 0: recovered centre node W^C (inverse tensor Simpson rule in conservative
// variables).
template <class T>
void recover_centres(Grid<T>& G, int nthreads) {
    G.C.assign(G.N(), Prim<T>{});
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int j = 0; j < G.ny; ++j)
        for (int i = 0; i < G.nx; ++i) {
            T Uc[4], U[4];
            const Prim<T> corners[4] = {G.node(NV, i, j), G.node(NV, i + 1, j), G.node(NV, i, j + 1), G.node(NV, i + 1, j + 1)};
            const Prim<T> edges[4] = {G.node(NEH, i, j), G.node(NEH, i, j + 1), G.node(NEV, i, j), G.node(NEV, i + 1, j)};
            T sc[4] = {0.0, 0.0, 0.0, 0.0}, se[4] = {0.0, 0.0, 0.0, 0.0};
            for (int c = 0; c < 4; ++c) {
                cons_of(corners[c], G.gamma, U);
                for (int k = 0; k < 4; ++k) sc[k] += U[k];
                cons_of(edges[c], G.gamma, U);
                for (int k = 0; k < 4; ++k) se[k] += U[k];
            }
            for (int k = 0; k < 4; ++k)
                Uc[k] = 2.25 * (G.at(k, i, j) - sc[k] / 36.0 - se[k] / 9.0);
            G.C[(int64_t)j * G.nx + i] = prim_of(Uc, G.gamma);
        }
}

// Steps 1-2 of Sec. 6.1 for one node: freeze (rho_K, c_K), apply the node-centred
// exact acoustic operator for duration tau, and return the physical increments
// (du, dv, dp).  Also reports r_K = c_K tau / h.
template <class T>
void node_increment(const Grid<T>& G, int fam, int i, int j, double tau, T inc[3], double* r_out) {
    Prim<T> WK = G.node(fam, i, j);
    T c = std::sqrt(G.gamma * WK.p / WK.r);
    T Z = WK.r * c;
    T r = c * tau / G.h;
    if (r_out) *r_out = re(r);
    const NodeDef& nd = kNodes[fam];
    T acc[3] = {0.0, 0.0, 0.0};
    for (int w = 0; w < nd.nw; ++w) {
        const WedgeDef& wd = nd.w[w];
        int ci = i + wd.dci, cj = j + wd.dcj;
        Prim<T> n[3][3];
        G.cell_nodes(ci, cj, n);
        T f[3][3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                f[0][a][b] = n[a][b].p / Z;
                f[1][a][b] = n[a][b].u;
                f[2][a][b] = n[a][b].v;
            }
        // lower-left node of the cell relative to K, in units of h
        double X0 = (double)wd.dci - nd.ox, Y0 = (double)wd.dcj - nd.oy;
        T out[3];
        wedge_apply(wd.mask, X0, Y0, f, r, out);
        for (int k = 0; k < 3; ++k) acc[k] += out[k];
    }
    inc[0] = acc[1] - WK.u;
    inc[1] = acc[2] - WK.v;
    inc[2] = Z * acc[0] - WK.p;
}

// Lagrange weights at -1, 0, 1 (Sec. 4: l_-(s) = s(s-1)/2, l_0 = 1 - s^2, l_+ = s(s+1)/2).
template <class T>
void lag3(T s, T l[3]) {
    l[0] = 0.5 * s * (s - 1.0);
    l[1] = 1.0 - s * s;
    l[2] = 0.5 * s * (s + 1.0);
}

// Locate a point given as (integer base + fractional offset) in cell units:
// containing cell index and local coordinate xi in [-1, 1].
template <class T>
void locate(int base, T off, int* cell, T* xi) {
    double fl = std::floor(re(off));
    *cell = base + (int)fl;
    *xi = 2.0 * (off - fl) - 1.0;
}

template <class T>
struct Increments {
    int nx, ny;
    std::vector<T> d;   // [fam 0..3][var 0..2][j][i]
    T get(int fam, int var, int i, int j) const {
        return d[((int64_t)(fam * 3 + var) * ny + wrap(j, ny)) * nx + wrap(i, nx)];
    }
};

// Nine node increments of cell (ci, cj) for variable `var`, [x-node][y-node].
template <class T>
void cell_incs(const Increments<T>& D, int var, int ci, int cj, T f[3][3]) {
    f[0][0] = D.get(NV, var, ci, cj);      f[1][0] = D.get(NEH, var, ci, cj);      f[2][0] = D.get(NV, var, ci + 1, cj);
    f[0][1] = D.get(NEV, var, ci, cj);     f[1][1] = D.get(NC, var, ci, cj);       f[2][1] = D.get(NEV, var, ci + 1, cj);
    f[0][2] = D.get(NV, var, ci, cj + 1);  f[1][2] = D.get(NEH, var, ci, cj + 1);  f[2][2] = D.get(NV, var, ci + 1, cj + 1);
}

template <class T>
T q2(const T f[3][3], const T lx[3], const T ly[3]) {
    T s = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s += lx[a] * ly[b] * f[a][b];
    return s;
}

enum Status { ST_OK = 0, ST_ACOUSTIC_CFL = 1, ST_FOOT = 2, ST_NONPHYSICAL = 3 };

// Point update of Sec. 6.1 steps 3-4 for target family fam in {V, Ev, Eh} at (i, j).
// scheme 0: transported increments (eq. transported-update); 1: additive RB
// (eq. barsukow-additive).  feet (optional): foot displacement in cell units.
template <class T>
Prim<T> point_update(const Grid<T>& G, const Increments<T>& D, int fam, int i, int j, double tau,
                     int scheme, int* status, double foot_out[2]) {
    const NodeDef& nd = kNodes[fam];
    Prim<T> WP = G.node(fam, i, j);
    const double lam = tau / G.h;
    // first Picard step: the reconstruction at a node equals the node value
    T fx1 = nd.ox - lam * WP.u, fy1 = nd.oy - lam * WP.v;
    int ci, cj;
    T xi, eta;
    locate(i, fx1, &ci, &xi);
    locate(j, fy1, &cj, &eta);
    Prim<T> n[3][3];
    G.cell_nodes(ci, cj, n);
    T lx[3], ly[3];
    lag3(xi, lx);
    lag3(eta, ly);
    T fu[3][3], fv[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) { fu[a][b] = n[a][b].u; fv[a][b] = n[a][b].v; }
    T u1 = q2(fu, lx, ly), v1 = q2(fv, lx, ly);
    // second Picard step, from P
    T fx = nd.ox - lam * u1, fy = nd.oy - lam * v1;
    if (foot_out) { foot_out[0] = re(fx) - nd.ox; foot_out[1] = re(fy) - nd.oy; }
    if (std::fabs(re(fx) - nd.ox) >= 1.0 || std::fabs(re(fy) - nd.oy) >= 1.0 ||
        std::fabs(re(fx1) - nd.ox) >= 1.0 || std::fabs(re(fy1) - nd.oy) >= 1.0)
        *status = ST_FOOT;
    locate(i, fx, &ci, &xi);
    locate(j, fy, &cj, &eta);
    G.cell_nodes(ci, cj, n);
    lag3(xi, lx);
    lag3(eta, ly);
    T fr[3][3], fp[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            fr[a][b] = n[a][b].r; fu[a][b] = n[a][b].u; fv[a][b] = n[a][b].v; fp[a][b] = n[a][b].p;
        }
    Prim<T> Wf{q2(fr, lx, ly), q2(fu, lx, ly), q2(fv, lx, ly), q2(fp, lx, ly)};
    T du, dv, dp, c2;
    if (scheme == 0) {
        T f[3][3];
        cell_incs(D, 0, ci, cj, f); du = q2(f, lx, ly);
        cell_incs(D, 1, ci, cj, f); dv = q2(f, lx, ly);
        cell_incs(D, 2, ci, cj, f); dp = q2(f, lx, ly);
        c2 = G.gamma * Wf.p / Wf.r;                    // c^2 at the foot
    } else {
        du = D.get(fam, 0, i, j);
        dv = D.get(fam, 1, i, j);
        dp = D.get(fam, 2, i, j);
        c2 = G.gamma * WP.p / WP.r;                    // frozen c^2 at the node P
    }
    return Prim<T>{Wf.r + dp / c2, Wf.u + du, Wf.v + dv, Wf.p + dp};
}

template <class T>
void flux_x(const Prim<T>& w, double g, T F[4]) {
    T E = w.p / (g - 1.0) + 0.5 * w.r * (w.u * w.u + w.v * w.v);
    F[0] = w.r * w.u;
    F[1] = w.r * w.u * w.u + w.p;
    F[2] = w.r * w.u * w.v;
    F[3] = w.u * (E + w.p);
}

template <class T>
void flux_y(const Prim<T>& w, double g, T F[4]) {
    T E = w.p / (g - 1.0) + 0.5 * w.r * (w.u * w.u + w.v * w.v);
    F[0] = w.r * w.v;
    F[1] = w.r * w.u * w.v;
    F[2] = w.r * w.v * w.v + w.p;
    F[3] = w.v * (E + w.p);
}

template <class T>
void compute_increments(const Grid<T>& G, double tau, Increments<T>& D, double* rmax, int nthreads) {
    D.nx = G.nx; D.ny = G.ny;
    D.d.assign((size_t)12 * G.N(), T(0.0));
    double rm = 0.0;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(max : rm)
    for (int j = 0; j < G.ny; ++j)
        for (int i = 0; i < G.nx; ++i)
            for (int fam = 0; fam < 4; ++fam) {
                T inc[3];
                double r;
                node_increment(G, fam, i, j, tau, inc, &r);
                if (r > rm) rm = r;
                for (int v = 0; v < 3; ++v) D.d[((int64_t)(fam * 3 + v) * G.ny + j) * G.nx + i] = inc[v];
            }
    *rmax = rm;
}

template <class T>
bool physical(const Grid<T>& G) {
    for (int j = 0; j < G.ny; ++j)
        for (int i = 0; i < G.nx; ++i)
            for (int fam = 0; fam < 4; ++fam) {
                Prim<T> w = G.node(fam, i, j);
                if (!(re(w.r) > 0.0) || !(re(w.p) > 0.0)) return false;
            }
    return true;
}

// One full step of Sec. 6.1.  in/out: 16 planes (ny, nx).
template <class T>
int step(int nx, int ny, double h, double gamma, double dt, int scheme, int nthreads,
         const T* in, T* out) {
    Grid<T> G{nx, ny, h, gamma, in, {}};
    recover_centres(G, nthreads);
    if (!physical(G)) return ST_NONPHYSICAL;
    const int64_t N = G.N();
    // point values at sigma = 1/2 and sigma = 1
    std::vector<Prim<T>> Pn[2][3];
    int status = ST_OK;
    for (int st = 0; st < 2; ++st) {
        double tau = (st == 0) ? 0.5 * dt : dt;
        Increments<T> D;
        double rmax;
        compute_increments(G, tau, D, &rmax, nthreads);
        if (st == 1 && rmax > 0.5) return ST_ACOUSTIC_CFL;
        for (int fam = 0; fam < 3; ++fam) Pn[st][fam].assign(N, Prim<T>{});
        int stt = ST_OK;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(max : stt)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (int fam = 0; fam < 3; ++fam) {
                    int s = ST_OK;
                    Pn[st][fam][(int64_t)j * nx + i] = point_update(G, D, fam, i, j, tau, scheme, &s, nullptr);
                    if (s > stt) stt = s;
                }
        if (stt > status) status = stt;
    }
    if (status != ST_OK) return status;
    auto point = [&](int st, int fam, int i, int j) -> Prim<T> {
        if (st == 0) return G.node(fam, i, j);
        return Pn[st - 1][fam][(int64_t)wrap(j, ny) * nx + wrap(i, nx)];
    };
    // Time-integrated Simpson fluxes: Fh[i,j] on the vertical edge x = x_i,
    // Gh[i,j] on the horizontal edge y = y_j.
    std::vector<T> Fh((size_t)4 * N), Gh((size_t)4 * N);
    const double wt[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            T Ft[4] = {0.0, 0.0, 0.0, 0.0}, Gt[4] = {0.0, 0.0, 0.0, 0.0};
            for (int st = 0; st < 3; ++st) {
                T a[4], b[4], c[4], Fs[4], Gs[4];
                flux_x(point(st, NV, i, j), gamma, a);
                flux_x(point(st, NEV, i, j), gamma, b);
                flux_x(point(st, NV, i, j + 1), gamma, c);
                for (int k = 0; k < 4; ++k) Fs[k] = (a[k] + 4.0 * b[k] + c[k]) / 6.0;
                flux_y(point(st, NV, i, j), gamma, a);
                flux_y(point(st, NEH, i, j), gamma, b);
                flux_y(point(st, NV, i + 1, j), gamma, c);
                for (int k = 0; k < 4; ++k) Gs[k] = (a[k] + 4.0 * b[k] + c[k]) / 6.0;
                for (int k = 0; k < 4; ++k) { Ft[k] += wt[st] * Fs[k]; Gt[k] += wt[st] * Gs[k]; }
            }
            for (int k = 0; k < 4; ++k) {
                Fh[(int64_t)k * N + (int64_t)j * nx + i] = Ft[k];
                Gh[(int64_t)k * N + (int64_t)j * nx + i] = Gt[k];
            }
        }
    const double lam = dt / h;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int64_t c = (int64_t)j * nx + i;
            int64_t ip = (int64_t)j * nx + wrap(i + 1, nx), jp = (int64_t)wrap(j + 1, ny) * nx + i;
            for (int k = 0; k < 4; ++k)
                out[(int64_t)k * N + c] = in[(int64_t)k * N + c] - lam * (Fh[k * N + ip] - Fh[k * N + c]) -
                                          lam * (Gh[k * N + jp] - Gh[k * N + c]);
            for (int fam = 0; fam < 3; ++fam) {
                const Prim<T>& w = Pn[1][fam][c];
                int b = 4 + 4 * fam;
                out[(int64_t)b * N + c] = w.r;
                out[(int64_t)(b + 1) * N + c] = w.u;
                out[(int64_t)(b + 2) * N + c] = w.v;
                out[(int64_t)(b + 3) * N + c] = w.p;
            }
        }
    return ST_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points (ctypes).  State arrays: 16 planes of ny*nx doubles, x fastest.
// ---------------------------------------------------------------------------
extern "C" {

int orc_num_threads_default() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_monomial_block(int a, int b, int quad_mask, double* C) { monomial_block(a, b, quad_mask, C); }

// Apply one wedge of node type `fam` (wedge index w as listed above) to a cell's
// 3x3 nodal (pi, u, v) data f[var][x-node][y-node]; out = (pi, u, v) contribution.
int orc_wedge_apply(int fam, int w, double r, const double* f, double* out) {
    if (fam < 0 || fam > 3 || w < 0 || w >= kNodes[fam].nw) return -1;
    const WedgeDef& wd = kNodes[fam].w[w];
    double ff[3][3][3];
    std::memcpy(ff, f, sizeof(ff));
    wedge_apply<double>(wd.mask, (double)wd.dci - kNodes[fam].ox, (double)wd.dcj - kNodes[fam].oy, ff, r, out);
    return 0;
}

int orc_centres(int nx, int ny, double h, double gamma, const double* in, double* out4) {
    Grid<double> G{nx, ny, h, gamma, in, {}};
    recover_centres(G, 1);
    int64_t N = G.N();
    for (int64_t c = 0; c < N; ++c) {
        out4[c] = G.C[c].r; out4[N + c] = G.C[c].u; out4[2 * N + c] = G.C[c].v; out4[3 * N + c] = G.C[c].p;
    }
    return 0;
}

// Increments (du, dv, dp) at V, Ev, Eh, C for duration tau: out has 12 planes
// ordered [family][var].  Returns max r_K.
double orc_increments(int nx, int ny, double h, double gamma, double tau, int nthreads,
                      const double* in, double* out12) {
    Grid<double> G{nx, ny, h, gamma, in, {}};
    recover_centres(G, nthreads);
    Increments<double> D;
    double rmax;
    compute_increments(G, tau, D, &rmax, nthreads);
    std::memcpy(out12, D.d.data(), sizeof(double) * D.d.size());
    return rmax;
}

// Feet of every target for duration tau: out has 6 planes (dx, dy) for V, Ev, Eh,
// the displacement from the target in cell units.  Also the transported point
// values (12 planes) in pts.
int orc_feet(int nx, int ny, double h, double gamma, double tau, int scheme, const double* in,
             double* feet6, double* pts12) {
    Grid<double> G{nx, ny, h, gamma, in, {}};
    recover_centres(G, 1);
    Increments<double> D;
    double rmax;
    compute_increments(G, tau, D, &rmax, 1);
    int64_t N = G.N();
    int status = ST_OK;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int fam = 0; fam < 3; ++fam) {
                double ft[2];
                Prim<double> w = point_update(G, D, fam, i, j, tau, scheme, &status, ft);
                int64_t c = (int64_t)j * nx + i;
                feet6[(2 * fam) * N + c] = ft[0];
                feet6[(2 * fam + 1) * N + c] = ft[1];
                pts12[(4 * fam) * N + c] = w.r; pts12[(4 * fam + 1) * N + c] = w.u;
                pts12[(4 * fam + 2) * N + c] = w.v; pts12[(4 * fam + 3) * N + c] = w.p;
            }
    return status;
}

int orc_step(int nx, int ny, double h, double gamma, double dt, int scheme, int nthreads,
             const double* in, double* out) {
    return step<double>(nx, ny, h, gamma, dt, scheme, nthreads, in, out);
}

// nsteps steps, ping-ponging through a scratch copy; result in out.
int orc_run(int nx, int ny, double h, double gamma, double dt, int scheme, int nthreads, int nsteps,
            const double* in, double* out) {
    size_t n = (size_t)16 * nx * ny;
    std::vector<double> a(in, in + n), b(n);
    for (int s = 0; s < nsteps; ++s) {
        int st = step<double>(nx, ny, h, gamma, dt, scheme, nthreads, a.data(), b.data());
        if (st) return st;
        a.swap(b);
    }
    std::memcpy(out, a.data(), n * sizeof(double));
    return 0;
}

// Complex-step directional derivative: out = step(in), jvp = d step(in + e dir)/de.
int orc_step_jvp(int nx, int ny, double h, double gamma, double dt, int scheme, int nthreads,
                 const double* in, const double* dir, double* out, double* jvp) {
    const double e = 1e-30;
    size_t n = (size_t)16 * nx * ny;
    std::vector<cplx> a(n), b(n);
    for (size_t k = 0; k < n; ++k) a[k] = cplx(in[k], e * dir[k]);
    int st = step<cplx>(nx, ny, h, gamma, dt, scheme, nthreads, a.data(), b.data());
    for (size_t k = 0; k < n; ++k) { out[k] = b[k].real(); jvp[k] = b[k].imag() / e; }
    return st;
}

// Diagnostics of the state (Sec. 6 opening paragraph; Sec. 3 conservation; the
// vorticity integrals of the low-Mach shear experiment, Sec. 6):
// out = {mass, momx, momy, energy, entropy, min_rho, min_p, max(|u|+c), max c dt/h,
//        int omega dA, int omega^2 dA}.
// omega = dv/dx - du/dy of the continuous piecewise-Q2 velocity reconstruction (the
// nine nodal values of each cell, recovered centre included); per cell both integrals
// use the 3x3 Gauss-Legendre rule, exact for omega (degree <= 2 in each direction) and
// omega^2 (degree <= 4).
int orc_diagnostics(int nx, int ny, double h, double gamma, double dt, const double* in, double* out) {
    Grid<double> G{nx, ny, h, gamma, in, {}};
    recover_centres(G, 1);
    int64_t N = G.N();
    double tot[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k)
        for (int64_t c = 0; c < N; ++c) tot[k] += in[k * N + c];
    double ent = 0.0, minr = 1e300, minp = 1e300, maxs = 0.0, maxr = 0.0, vort = 0.0, enst = 0.0;
    const double wq[3] = {1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0};
    // Gauss-Legendre on [-1, 1]: nodes and weights
    const double gs[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)}, gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    // Lagrange basis on the nodes -1, 0, 1 and its derivative
    auto lag = [](double t, double L[3], double dL[3]) {
        L[0] = 0.5 * t * (t - 1.0); L[1] = 1.0 - t * t; L[2] = 0.5 * t * (t + 1.0);
        dL[0] = t - 0.5;            dL[1] = -2.0 * t;   dL[2] = t + 0.5;
    };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            Prim<double> n[3][3];
            G.cell_nodes(i, j, n);
            double e = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const Prim<double>& w = n[a][b];
                    e += wq[a] * wq[b] * w.r * std::log(w.p / std::pow(w.r, gamma));
                }
            ent -= e;
            // x = x_i + (1 + xi) h / 2: d/dx = (2 / h) d/dxi; the cell's area element h^2 / 4
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) {
                    double Lx[3], dLx[3], Ly[3], dLy[3];
                    lag(gs[p], Lx, dLx);
                    lag(gs[q], Ly, dLy);
                    double dvdx = 0.0, dudy = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            dvdx += dLx[a] * Ly[b] * n[a][b].v;
                            dudy += Lx[a] * dLy[b] * n[a][b].u;
                        }
                    const double om = (2.0 / h) * (dvdx - dudy);
                    vort += gw[p] * gw[q] * om;
                    enst += gw[p] * gw[q] * om * om;
                }
            for (int fam = 0; fam < 4; ++fam) {
                Prim<double> w = G.node(fam, i, j);
                double c = std::sqrt(gamma * w.p / w.r);
                minr = std::fmin(minr, w.r);
                minp = std::fmin(minp, w.p);
                maxs = std::fmax(maxs, std::sqrt(w.u * w.u + w.v * w.v) + c);
                maxr = std::fmax(maxr, c * dt / h);
            }
        }
    double A = h * h;
    out[0] = tot[0] * A; out[1] = tot[1] * A; out[2] = tot[2] * A; out[3] = tot[3] * A;
    out[4] = ent * A; out[5] = minr; out[6] = minp; out[7] = maxs; out[8] = maxr;
    out[9] = vort * A * 0.25; out[10] = enst * A * 0.25;
    return 0;
}

}  // extern "C"
