"""Test helpers: piecewise-Q2 fields on a grid and exact solutions of the frozen
linear acoustic system, written independently of the oracle (numpy only).

Units: lengths in cells (h = 1); the frozen system is u_t + c grad(pi) = 0,
pi_t + c div(u) = 0 (Sec. 3.1, eq. lin-ac-u / lin-ac-pi).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def lag(s):
    """Lagrange basis at -1, 0, 1 and its first two derivatives (w.r.t. s)."""
    s = np.asarray(s, dtype=float)
    L = np.stack([0.5 * s * (s - 1), 1 - s * s, 0.5 * s * (s + 1)])
    dL = np.stack([s - 0.5, -2 * s, s + 0.5])
    d2L = np.stack([np.ones_like(s), -2 * np.ones_like(s), np.ones_like(s)])
    return L, dL, d2L


class PiecewiseQ2:
    """A continuous piecewise-Q2 scalar field on the integer grid, defined by its
    values on the half-integer node lattice: node (a, b) sits at (a/2, b/2)."""

    def __init__(self, nodes: np.ndarray, ox: int = 0, oy: int = 0):
        self.n = np.asarray(nodes, float)    # shape (2*ncx+1, 2*ncy+1), [x][y]
        self.ox, self.oy = ox, oy            # lattice node (0,0) sits at (ox, oy)

    def _cell(self, x, y, cx=None, cy=None):
        X = np.asarray(x, float) - self.ox
        Y = np.asarray(y, float) - self.oy
        ci = np.floor(X).astype(int) if cx is None else np.full(np.shape(X), cx, dtype=int) - self.ox
        cj = np.floor(Y).astype(int) if cy is None else np.full(np.shape(Y), cy, dtype=int) - self.oy
        xi = 2 * (X - ci) - 1
        eta = 2 * (Y - cj) - 1
        return ci, cj, xi, eta

    def eval(self, x, y, d=(0, 0), cx=None, cy=None):
        """Value or derivative d=(dx, dy) order in x, y (each <= 2), physical units.
        cx, cy force the cell (for one-sided limits on a grid line)."""
        ci, cj, xi, eta = self._cell(x, y, cx, cy)
        Lx = lag(xi)[d[0]] * (2.0 ** d[0])
        Ly = lag(eta)[d[1]] * (2.0 ** d[1])
        out = np.zeros(np.shape(xi))
        for a in range(3):
            for b in range(3):
                out = out + Lx[a] * Ly[b] * self.n[2 * ci + a, 2 * cj + b]
        return out


def poly2d_eval(c, x, y):
    """c[a][b] coefficient of x^a y^b."""
    out = 0.0
    for a in range(c.shape[0]):
        for b in range(c.shape[1]):
            out = out + c[a, b] * x ** a * y ** b
    return out


def poly2d_dx(c):
    out = np.zeros_like(c)
    out[:-1, :] = c[1:, :] * np.arange(1, c.shape[0])[:, None]
    return out


def poly2d_dy(c):
    out = np.zeros_like(c)
    out[:, :-1] = c[:, 1:] * np.arange(1, c.shape[1])[None, :]
    return out


def ck_solution(cpi, cu, cv, c, t, x, y):
    """Exact solution at (x, y, t) of the frozen acoustic system for polynomial data
    by the terminating Cauchy-Kowalevskaya (Taylor-in-time) series
    w(t) = sum_k t^k/k! L^k w0, with L(pi, u, v) = -c (u_x + v_y, pi_x, pi_y)."""
    P, U, V = (np.array(a, float) for a in (cpi, cu, cv))
    res = [0.0, 0.0, 0.0]
    fact = 1.0
    for k in range(0, 9):
        if k > 0:
            fact *= k
        coef = t ** k / fact
        res[0] += coef * poly2d_eval(P, x, y)
        res[1] += coef * poly2d_eval(U, x, y)
        res[2] += coef * poly2d_eval(V, x, y)
        P, U, V = -c * (poly2d_dx(U) + poly2d_dy(V)), -c * poly2d_dx(P), -c * poly2d_dy(P)
    return res


def _gl(n, a, b):
    g, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * g + 0.5 * (b + a), 0.5 * (b - a) * w


def poisson_node(fpi: PiecewiseQ2, fu: PiecewiseQ2, fv: PiecewiseQ2, K, lines, c, t, nq=28):
    """Exact frozen-acoustic (pi, u, v) at node K after time t for continuous
    piecewise-Q2 data, from the Poisson formula of the 2-D wave equation,
    integrated numerically over the disk |y - K| < ct split along the grid lines
    through K.  lines = (xline, yline): whether x = K_x / y = K_y is a cell face.
      pi(K, t) = d/dt (t S_t[pi0]) - c t S_t[div u0]
      u(K, t)  = u0(K) - c grad Pi,  Pi = t S_t[pi0] - c int_0^t s S_s[div u0] ds,
    with S_t[f] = (1/2pi) int_{|z|<1} f(K + c t z) (1 - |z|^2)^{-1/2} dz and the
    distributional gradient of div u0 (jumps across the face lines give line terms).
    """
    Kx, Ky = K
    R = c * t
    # disk quadrature: z = sin(phi) (cos th, sin th); weight rho drho/sqrt(1-rho^2) = sin(phi) dphi
    ph, wph = _gl(nq, 0.0, 0.5 * math.pi)
    pts, wts = [], []
    for q in range(4):
        th, wth = _gl(nq, q * 0.5 * math.pi, (q + 1) * 0.5 * math.pi)
        PH, TH = np.meshgrid(ph, th, indexing="ij")
        W = np.outer(wph, wth) * np.sin(PH)
        pts.append((np.sin(PH) * np.cos(TH), np.sin(PH) * np.sin(TH)))
        wts.append(W)
    zx = np.concatenate([p[0].ravel() for p in pts])
    zy = np.concatenate([p[1].ravel() for p in pts])
    wz = np.concatenate([w.ravel() for w in wts]) / (2 * math.pi)

    def S(f, s, d=(0, 0)):
        return np.sum(wz * f.eval(Kx + c * s * zx, Ky + c * s * zy, d))

    def Sgrad_dot_z(f, s):
        X, Y = Kx + c * s * zx, Ky + c * s * zy
        return np.sum(wz * (f.eval(X, Y, (1, 0)) * zx + f.eval(X, Y, (0, 1)) * zy))

    def Sdiv(s, d=(0, 0)):
        X, Y = Kx + c * s * zx, Ky + c * s * zy
        return np.sum(wz * (fu.eval(X, Y, (1 + d[0], d[1])) + fv.eval(X, Y, (d[0], 1 + d[1]))))

    pi = S(fpi, t) + t * c * Sgrad_dot_z(fpi, t) - c * t * Sdiv(t)

    # line terms of grad(div u0): jumps of g = div u0 across x = Kx and y = Ky
    phl, wphl = [], []
    for a, b in ((0.0, 0.5 * math.pi), (0.5 * math.pi, math.pi)):
        p_, w_ = _gl(nq, a, b)
        phl.append(p_)
        wphl.append(w_)
    phl = np.concatenate(phl)
    wphl = np.concatenate(wphl) / (2 * math.pi)

    def g_at(X, Y, cx=None, cy=None):
        return fu.eval(X, Y, (1, 0), cx, cy) + fv.eval(X, Y, (0, 1), cx, cy)

    def J(s):
        jx = jy = 0.0
        eta = np.cos(phl)                    # z2 = cos(phi), weight dphi
        if lines[0]:
            Y = Ky + c * s * eta
            jx = np.sum(wphl * (g_at(np.full_like(Y, Kx), Y, cx=int(Kx)) -
                                g_at(np.full_like(Y, Kx), Y, cx=int(Kx) - 1)))
        if lines[1]:
            X = Kx + c * s * eta
            jy = np.sum(wphl * (g_at(X, np.full_like(X, Ky), cy=int(Ky)) -
                                g_at(X, np.full_like(X, Ky), cy=int(Ky) - 1)))
        return jx, jy

    sg, wsg = _gl(12, 0.0, t)
    int_x = int_y = 0.0
    for s, w in zip(sg, wsg):
        jx, jy = J(s)
        int_x += w * (s * Sdiv(s, (1, 0)) + jx / c)
        int_y += w * (s * Sdiv(s, (0, 1)) + jy / c)
    gPx = t * S(fpi, t, (1, 0)) - c * int_x
    gPy = t * S(fpi, t, (0, 1)) - c * int_y
    u = fu.eval(np.array(Kx), np.array(Ky)) - c * gPx
    v = fv.eval(np.array(Kx), np.array(Ky)) - c * gPy
    return np.array([float(pi), float(u), float(v)])
