"""Foot-centred exact frozen-acoustic point update (App. C; Sec. 4, paragraph on an
exact frozen acoustic update) -- TEST INFRASTRUCTURE ONLY: an analytical reference
for the point update, slow by design (the paper quotes roughly a thousand times the
cost of the node-centred update for its closed-form version).

For a target P and a duration tau in {dt/2, dt} (App. C, eq. fc-foot-freeze):
  * the material foot F by the two Picard stages of the transported update (taken
    from the C++ oracle's foot computation),
  * the frozen state W_* = W_h^n(F) (the Q2 reconstruction at F), c_* = sqrt(gamma
    p_* / rho_*), Z_* = rho_* c_*, R = c_* tau,
  * the compact footprint condition |delta_x| + R < h/2, |delta_y| + R < h/2 with
    delta = F - P (eq. fc-half-footprint),
  * the exact solution at F after tau of the frozen acoustic system
    pi_t + c_* div u = 0, u_t + c_* grad pi = 0 with pi = p / Z_*, for the continuous
    piecewise-Q2 data of the cells the disk of radius R about F touches,
  * p^A = Z_* pi^A, and rho^A from the linear closure rho_h(F) + (p^A - p_h(F)) / c_*^2
    (the closure of the transported update) or, optionally, the isentropic one
    rho_h(F) (p^A / p_h(F))^(1 / gamma).
The new point values at n + 1/2 and n + 1 then enter the same space-time Simpson
fluxes and conservative average update as the transported update (Sec. 3,
eq. af-average-update).

The exact solution is written with spherical means of the 2-D wave equation, in
cell units (lengths / h) with r = c_* s / h:
    M_r[f](F) = (1 / 2 pi) int_{|z| < 1} f(F + r z) (1 - |z|^2)^(-1/2) dz
(the projected-sphere weight of App. C), g = div u_0,
    pi(F)  = M_R[pi_0] + R M_R[z . grad pi_0] - R M_R[g],
    u(F)   = u_0(F) - R M_R[grad pi_0] + int_0^R r M_r[grad g] dr,
where grad g is the distributional gradient: g jumps across the grid lines that the
data's cells share, and each crossing line adds the chord term
    (1 / (2 pi r)) int_0^pi [g](point of the chord at angle phi) dphi   (normal n).
The paper evaluates these integrals in closed form from full-disk, single-cap and
double-cap moments (eq. fc-moment-families, eq. fc-cap-moments, eq. fc-role-rows).
Here they are integrated numerically.  The history term is first rewritten exactly as
one integral over the disk of radius R (see exact_acoustic), which needs neither the
radius integral nor the chord terms; history_by_radius keeps the form above as a
cross-check.  The disk integrals are split exactly along the grid lines that cut
the disk: in polar coordinates about F with rho = sin(psi) (which absorbs the
weight), the angle split where a grid line becomes tangent to the circle or passes
through a corner, the radius split where each ray crosses a line, and the radius
integral split at every fragment birth radius; angle and radius pieces use nodes
clustered quadratically at both ends (which absorbs the square-root behaviour at a
tangency and at the birth of a cap).  Every piece is then a smooth integrand and
Gauss-Legendre converges to round-off.
"""
from __future__ import annotations

import math

import numpy as np

from . import ref

NQ_THETA = 32      # Gauss points per angular piece
NQ_RHO = 10        # per radial piece
NQ_R = 12          # per piece of the history integral in r
NQ_CHORD = 12      # per piece of a chord integral


def _gl(n):
    return np.polynomial.legendre.leggauss(n)


_GL = {}


def gl(n, a, b):
    if n not in _GL:
        _GL[n] = _gl(n)
    x, w = _GL[n]
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def gl_ends(n, a, b):
    """Gauss-Legendre in s on [0, 1] with x = a + (b - a) (1 - cos(pi s)) / 2: the nodes
    cluster quadratically at both ends, so that an integrand behaving like the square
    root of the distance to an end (a cap being born, a line becoming tangent to the
    circle) becomes smooth in s."""
    s, ws = gl(n, 0.0, 1.0)
    x = a + 0.5 * (b - a) * (1.0 - np.cos(math.pi * s))
    return x, ws * 0.5 * (b - a) * math.pi * np.sin(math.pi * s)


# ---------------------------------------------------------------------------------
# Continuous piecewise-Q2 fields of a state (Sec. 2; Sec. 4, cellwise Q2 reconstruction)
# ---------------------------------------------------------------------------------
class Q2Lattice:
    """Nodal values of one primitive variable on the half-integer lattice of a
    periodic nx x ny grid: node (a, b) sits at (a/2, b/2) in cell units, so that
    (2i, 2j) is V_ij, (2i, 2j+1) Ev_ij, (2i+1, 2j) Eh_ij and (2i+1, 2j+1) C_ij."""

    def __init__(self, nodes):
        self.n = np.asarray(nodes, float)     # [x-node][y-node], shape (2 nx, 2 ny)
        self.mx, self.my = self.n.shape

    @staticmethod
    def of_state(state, centres, k):
        """Variable k in (rho, u, v, p) of a (16, ny, nx) state and (4, ny, nx) centres."""
        ny, nx = state.shape[1:]
        L = np.empty((2 * nx, 2 * ny))
        L[0::2, 0::2] = state[4 + k].T
        L[0::2, 1::2] = state[8 + k].T
        L[1::2, 0::2] = state[12 + k].T
        L[1::2, 1::2] = centres[k].T
        return Q2Lattice(L)

    def eval(self, X, Y, d=(0, 0), ci=None, cj=None):
        """Value (or derivative of orders d in X, Y, each <= 2) at points (X, Y) in
        cell units; ci, cj force the cell (one-sided values on a grid line)."""
        X = np.asarray(X, float)
        Y = np.asarray(Y, float)
        ci = np.floor(X).astype(int) if ci is None else np.broadcast_to(np.asarray(ci), X.shape)
        cj = np.floor(Y).astype(int) if cj is None else np.broadcast_to(np.asarray(cj), Y.shape)
        s = 2.0 * (X - ci) - 1.0
        t = 2.0 * (Y - cj) - 1.0
        Lx = _lag(s, d[0])
        Ly = _lag(t, d[1])
        out = np.zeros(np.shape(X))
        for a in range(3):
            ia = (2 * ci + a) % self.mx
            for b in range(3):
                jb = (2 * cj + b) % self.my
                out = out + Lx[a] * Ly[b] * self.n[ia, jb]
        return out


def _lag(s, d):
    """Lagrange basis at -1, 0, 1 (local coordinate s = 2 (X - cell) - 1) or its d-th
    derivative with respect to X (d/dX = 2 d/ds)."""
    if d == 0:
        return [0.5 * s * (s - 1.0), 1.0 - s * s, 0.5 * s * (s + 1.0)]
    if d == 1:
        return [2.0 * (s - 0.5), 2.0 * (-2.0 * s), 2.0 * (s + 0.5)]
    one = np.ones_like(s)
    return [4.0 * one, -8.0 * one, 4.0 * one]


# ---------------------------------------------------------------------------------
# Spherical means over a disk split along the grid lines
# ---------------------------------------------------------------------------------
def _lines(c, r):
    """Integer grid lines k with |k - c| < r."""
    return [k for k in range(math.floor(c - r) + 1, math.ceil(c + r)) if abs(k - c) < r]


def disk_nodes(F, r):
    """Quadrature of M_r: points (X, Y), unit-disk positions (zx, zy) and weights
    (summing to 1 for f = 1), split so that every piece lies in one cell."""
    Fx, Fy = F
    vx, vy = _lines(Fx, r), _lines(Fy, r)
    # eight base pieces (Gauss-Legendre is not exact for trigonometric integrands; short
    # pieces reach round-off with few points), plus the geometric cuts
    cuts = [q * 0.25 * math.pi for q in range(9)]
    def tangency(lam, base):
        # the crossing radius lam / cos(theta - base) runs from 1 (tangent) to |lam| over
        # an angle of order |lam| next to each tangency: cuts graded towards it
        a = math.acos(min(1.0, abs(lam)))
        out = [base - a, base + a]
        for g in (0.25, 1.0, 4.0):
            d = g * abs(lam)
            if d < a:
                out += [base - a + d, base + a - d]
        return out

    for k in vx:
        lam = (k - Fx) / r
        cuts += tangency(lam, 0.0 if lam > 0 else math.pi)
    for k in vy:
        mu = (k - Fy) / r
        cuts += tangency(mu, 0.5 * math.pi if mu > 0 else 1.5 * math.pi)
    for kx in vx:
        for ky in vy:
            if (kx - Fx) ** 2 + (ky - Fy) ** 2 < r * r:
                cuts.append(math.atan2(ky - Fy, kx - Fx))
    cuts = sorted({c % (2.0 * math.pi) for c in cuts} | {0.0, 2.0 * math.pi})
    ZX, ZY, Ws = [], [], []
    for t0, t1 in zip(cuts[:-1], cuts[1:]):
        if t1 - t0 < 1e-15:
            continue
        th, wth = gl_ends(NQ_THETA, t0, t1)
        ct, st = np.cos(th), np.sin(th)
        # radii at which the rays of this piece cross each line: within a piece every
        # ray crosses the same lines in the same order (the cuts above)
        tm = 0.5 * (t0 + t1)
        cross = []
        for k in vx:
            lam = (k - Fx) / r
            if lam / math.cos(tm) > 0.0 and lam / math.cos(tm) < 1.0:
                cross.append(lam / ct)
        for k in vy:
            mu = (k - Fy) / r
            if mu / math.sin(tm) > 0.0 and mu / math.sin(tm) < 1.0:
                cross.append(mu / st)
        bounds = [np.zeros_like(th)] + sorted(np.arcsin(np.clip(cross, 0.0, 1.0)), key=lambda x: float(x[0]))
        bounds.append(np.full_like(th, 0.5 * math.pi))
        if NQ_RHO not in _GL:
            _GL[NQ_RHO] = _gl(NQ_RHO)
        xq, wq = _GL[NQ_RHO]
        for p0, p1 in zip(bounds[:-1], bounds[1:]):
            ps = 0.5 * (p1 - p0)[:, None] * xq[None, :] + 0.5 * (p1 + p0)[:, None]
            wps = 0.5 * (p1 - p0)[:, None] * wq[None, :]
            rho = np.sin(ps)
            ZX.append((rho * ct[:, None]).ravel())
            ZY.append((rho * st[:, None]).ravel())
            Ws.append((wth[:, None] * wps * rho / (2.0 * math.pi)).ravel())
    zx, zy, w = np.concatenate(ZX), np.concatenate(ZY), np.concatenate(Ws)
    return Fx + r * zx, Fy + r * zy, zx, zy, w


def chord_nodes(F, r):
    """Quadrature of the singular part of M_r[grad g] for g with jumps across the grid
    lines that cut the disk: a vertical line x = k contributes, along x,
        (1 / (2 pi r)) int_0^pi [g](k, F_y + r sqrt(1 - lambda^2) cos phi) dphi
    (the jump taken as right minus left), a horizontal line likewise along y.
    Returns points (X, Y), the cells on the two sides (ci, cj) and (ci', cj') such that
    the jump is g(X, Y; ci, cj) - g(X, Y; ci', cj'), weights and the axis (0: x, 1: y)."""
    Fx, Fy = F
    X, Y, CI, CJ, CI2, CJ2, W, AX = [], [], [], [], [], [], [], []
    for axis, (c0, c1) in enumerate(((Fx, Fy), (Fy, Fx))):
        for k in _lines(c0, r):
            lam = (k - c0) / r
            half = r * math.sqrt(max(0.0, 1.0 - lam * lam))
            # the chord's other coordinate runs over c1 + half cos(phi): split it where
            # it crosses the perpendicular grid lines
            cuts = [0.0, math.pi]
            for m in _lines(c1, half) if half > 0 else []:
                cuts.append(math.acos(max(-1.0, min(1.0, (m - c1) / half))))
            cuts = sorted(set(cuts))
            for p0, p1 in zip(cuts[:-1], cuts[1:]):
                if p1 - p0 < 1e-15:
                    continue
                ph, wph = gl(NQ_CHORD, p0, p1)
                other = c1 + half * np.cos(ph)
                line = np.full_like(other, float(k))
                oc = np.floor(other).astype(int)
                kk = np.full(len(ph), k)
                if axis == 0:
                    X.append(line); Y.append(other); CI.append(kk); CJ.append(oc); CI2.append(kk - 1); CJ2.append(oc)
                else:
                    X.append(other); Y.append(line); CI.append(oc); CJ.append(kk); CI2.append(oc); CJ2.append(kk - 1)
                W.append(wph / (2.0 * math.pi * r))
                AX.append(np.full(len(ph), axis))
    if not W:
        e = np.zeros(0)
        ei = np.zeros(0, dtype=int)
        return e, e, ei, ei, ei, ei, e, ei
    return tuple(np.concatenate(v) for v in (X, Y, CI, CJ, CI2, CJ2, W, AX))


def exact_acoustic(F, R, fpi, fu, fv):
    """(pi, u, v) at F after the frozen acoustic evolution over the radius R (cell
    units) from continuous piecewise-Q2 data pi_0 = fpi, u_0 = fu, v_0 = fv.

    The history term int_0^R r M_r[grad g] dr is taken as one disk integral:
    exchanging the order of integration turns it into (1 / 2 pi) int_{|y| < R}
    grad g(F + y) arccosh(R / |y|) dy, and integrating by parts piece by piece (the
    weight vanishes on the circle; the jump terms of the distributional gradient
    cancel the pieces' boundary terms along the grid lines) into
    (R / 2 pi) int_0^{2 pi} e_theta int_0^{pi/2} g(F + R sin(psi) e_theta) dpsi dtheta,
    i.e. R sum w g z / |z|^2 over the same nodes as M_R.  history_by_radius evaluates
    the original form (radius integral of spherical means plus chord terms) for the
    pins."""
    Fx, Fy = F
    X, Y, zx, zy, w = disk_nodes(F, R)
    pi0 = fpi.eval(X, Y)
    px, py = fpi.eval(X, Y, (1, 0)), fpi.eval(X, Y, (0, 1))
    g = fu.eval(X, Y, (1, 0)) + fv.eval(X, Y, (0, 1))
    pi = np.sum(w * pi0) + R * np.sum(w * (zx * px + zy * py)) - R * np.sum(w * g)
    z2 = zx * zx + zy * zy
    hist = np.array([R * np.sum(w * g * zx / z2), R * np.sum(w * g * zy / z2)])
    u = float(fu.eval(np.array(Fx), np.array(Fy))) - R * np.sum(w * px) + hist[0]
    v = float(fv.eval(np.array(Fx), np.array(Fy))) - R * np.sum(w * py) + hist[1]
    return np.array([float(pi), u, v])


def history_by_radius(F, R, fu, fv):
    """int_0^R r M_r[grad g] dr, g = div u_0, as written in App. C: spherical means of
    the regular part of grad g at Gauss radii (split at every radius where a line or a
    corner enters the disk) plus, for each grid line crossing the disk of radius r, the
    chord integral of the jump of g (the singular part of the distributional gradient).
    Converges more slowly than the form exact_acoustic uses where lines pass close to
    F (raise NQ_THETA, NQ_RHO, NQ_R)."""
    Fx, Fy = F
    def g_at(XX, YY, ci, cj):
        return fu.eval(XX, YY, (1, 0), ci, cj) + fv.eval(XX, YY, (0, 1), ci, cj)

    # int_0^R r M_r[grad g] dr, split at every birth radius of a fragment
    births = set()
    for k in _lines(Fx, R):
        births.add(abs(k - Fx))
    for k in _lines(Fy, R):
        births.add(abs(k - Fy))
    for kx in _lines(Fx, R):
        for ky in _lines(Fy, R):
            d = math.hypot(kx - Fx, ky - Fy)
            if d < R:
                births.add(d)
    edges = sorted({0.0, R} | {b for b in births if 0.0 < b < R})
    # all radii of the history integral at once: one field evaluation over the union
    # of their disk nodes, summed per radius
    radii, rw = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        rr, ww = gl_ends(NQ_R, a, b)
        radii += list(rr)
        rw += list(ww)
    XS, YS, WS, IDX = [], [], [], []
    CH = [[] for _ in range(8)]
    for q, r in enumerate(radii):
        Xr, Yr, _, _, wr = disk_nodes(F, r)
        XS.append(Xr)
        YS.append(Yr)
        WS.append(wr)
        IDX.append(np.full(len(wr), q))
        cn = chord_nodes(F, r)
        for m in range(7):
            CH[m].append(cn[m])
        CH[7].append(2 * q + cn[7])          # bin: radius q, axis
    Xa, Ya, Wa, Ia = np.concatenate(XS), np.concatenate(YS), np.concatenate(WS), np.concatenate(IDX)
    nr = len(radii)
    gx = np.bincount(Ia, Wa * (fu.eval(Xa, Ya, (2, 0)) + fv.eval(Xa, Ya, (1, 1))), nr)
    gy = np.bincount(Ia, Wa * (fu.eval(Xa, Ya, (1, 1)) + fv.eval(Xa, Ya, (0, 2))), nr)
    cX, cY, cI, cJ, cI2, cJ2, cW, cB = (np.concatenate(v) for v in CH)
    if len(cW):
        jump = g_at(cX, cY, cI, cJ) - g_at(cX, cY, cI2, cJ2)
        line = np.bincount(cB, cW * jump, 2 * nr).reshape(nr, 2)
    else:
        line = np.zeros((nr, 2))
    hist = np.zeros(2)
    for q, r in enumerate(radii):
        hist += rw[q] * r * (np.array([gx[q], gy[q]]) + line[q])
    return hist


# ---------------------------------------------------------------------------------
# The foot-centred point update and the step built on it
# ---------------------------------------------------------------------------------
FAM_OFFSET = {0: (0.0, 0.0), 1: (0.0, 0.5), 2: (0.5, 0.0)}     # V, Ev, Eh in cell units


class FootprintError(RuntimeError):
    """The disk about a foot leaves the compact footprint of eq. fc-half-footprint."""


def _prepare(state, h, gamma, tau):
    state = np.ascontiguousarray(state, float)
    C = ref.centres(state, h, gamma)
    feet, _, st = ref.feet(state, h, gamma, tau)
    if st == 2:
        raise FootprintError("a foot moved one cell or more")
    W = [Q2Lattice.of_state(state, C, k) for k in range(4)]
    return feet, W


def _target_value(feet, W, h, gamma, tau, fam, i, j, closure, check):
    """New point value (rho, u, v, p) of the target of family fam at (i, j)."""
    ox, oy = FAM_OFFSET[fam]
    dx, dy = feet[fam, 0, j, i], feet[fam, 1, j, i]
    Fx, Fy = i + ox + dx, j + oy + dy
    rho_s, u_s, v_s, p_s = (float(W[k].eval(np.array(Fx), np.array(Fy))) for k in range(4))
    c_s = math.sqrt(gamma * p_s / rho_s)
    Z_s = rho_s * c_s
    R = c_s * tau / h
    if check and (abs(dx) + R >= 0.5 or abs(dy) + R >= 0.5):
        raise FootprintError(f"target {fam} ({i}, {j}): |delta| + R >= h/2")
    fpi = Q2Lattice(W[3].n / Z_s)
    pi_a, u_a, v_a = exact_acoustic((Fx, Fy), R, fpi, W[1], W[2])
    p_a = Z_s * pi_a
    if closure == "linear":
        rho_a = rho_s + (p_a - p_s) / (c_s * c_s)
    else:
        rho_a = rho_s * (p_a / p_s) ** (1.0 / gamma)
    return np.array([rho_a, u_a, v_a, p_a])


def point_values(state, h, gamma, tau, closure="linear", check=True):
    """New point values (12, ny, nx) of all targets after tau by the foot-centred exact
    frozen-acoustic update; state absolute FP64 (16, ny, nx)."""
    _, ny, nx = np.shape(state)
    feet, W = _prepare(state, h, gamma, tau)
    out = np.empty((12, ny, nx))
    for fam in range(3):
        for j in range(ny):
            for i in range(nx):
                out[4 * fam:4 * fam + 4, j, i] = _target_value(feet, W, h, gamma, tau, fam, i, j, closure, check)
    return out


def point_values_at(state, h, gamma, tau, targets, closure="linear", check=True):
    """The same for a list of targets (fam, i, j) only: an array (len(targets), 4)."""
    feet, W = _prepare(state, h, gamma, tau)
    return np.array([_target_value(feet, W, h, gamma, tau, f, i, j, closure, check) for f, i, j in targets])


def _flux_x(W, g):
    r, u, v, p = W
    E = p / (g - 1.0) + 0.5 * r * (u * u + v * v)
    return np.stack([r * u, r * u * u + p, r * u * v, u * (E + p)])


def _flux_y(W, g):
    r, u, v, p = W
    E = p / (g - 1.0) + 0.5 * r * (u * u + v * v)
    return np.stack([r * v, r * u * v, r * v * v + p, v * (E + p)])


def step(state, h, gamma, dt, closure="linear", check=True):
    """One step with the foot-centred point update at tau = dt/2 and dt, then the
    space-time Simpson edge fluxes and the conservative average update (Sec. 3,
    eq. af-average-update; App. C, last sentence)."""
    state = np.ascontiguousarray(state, float)
    half = point_values(state, h, gamma, 0.5 * dt, closure, check)
    full = point_values(state, h, gamma, dt, closure, check)
    levels = [state[4:16], half, full]
    wt = [1.0 / 6.0, 4.0 / 6.0, 1.0 / 6.0]
    # time-Simpson fluxes at V (F and G), Ev (F), Eh (G)
    FV = sum(w * _flux_x(L[0:4], gamma) for w, L in zip(wt, levels))
    GV = sum(w * _flux_y(L[0:4], gamma) for w, L in zip(wt, levels))
    FE = sum(w * _flux_x(L[4:8], gamma) for w, L in zip(wt, levels))
    GE = sum(w * _flux_y(L[8:12], gamma) for w, L in zip(wt, levels))
    # spatial Simpson on the left edge x_i (V_ij, Ev_ij, V_i,j+1) and bottom edge y_j
    Fl = (FV + 4.0 * FE + np.roll(FV, -1, axis=1)) / 6.0
    Gb = (GV + 4.0 * GE + np.roll(GV, -1, axis=2)) / 6.0
    Fr = np.roll(Fl, -1, axis=2)
    Gt = np.roll(Gb, -1, axis=1)
    lam = dt / h
    out = np.empty_like(state)
    out[0:4] = state[0:4] - lam * ((Fr - Fl) + (Gt - Gb))
    out[4:16] = full
    return out


def run(state, h, gamma, dt, nsteps, closure="linear"):
    x = np.ascontiguousarray(state, float)
    for _ in range(nsteps):
        x = step(x, h, gamma, dt, closure)
    return x
