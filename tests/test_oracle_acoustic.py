"""Pins of the oracle's exact node-centred acoustic operator (App. D monomial block)
against facts fixed by the paper and by the mathematics:

* the explicit Ev-node stencils printed in App. B (golden fixture);
* the terminating Cauchy-Kowalevskaya series for globally Q2 data (the operator is
  exact, Sec. 3.1 / App. D: "a degree-four polynomial in r, not a Taylor
  approximation");
* d'Alembert's solution for one-dimensional data with a kink on a grid line;
* the Poisson formula of the 2-D wave equation for general continuous piecewise-Q2
  data around every node type (numerical quadrature, independent of the block).
"""
import math
import os
import re

import numpy as np
import pytest

from tests import q2field as qf

HERE = os.path.dirname(os.path.abspath(__file__))
GAMMA = 1.4


def load_appB():
    mats, cur = {}, None
    with open(os.path.join(HERE, "golden", "appB_ev_stencils.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            m = re.match(r"\[(\w+)\]", line)
            if m:
                cur = m.group(1)
                mats[cur] = []
                continue
            mats[cur].append([e.strip() for e in line.split(";")])
    return mats


APPB = load_appB()


def appB(name, nu):
    return np.array([[eval(e, {"nu": nu}) for e in row] for row in APPB[name]], dtype=float)


@pytest.mark.parametrize("nu", [0.0, 0.05, 0.17, 0.25, 0.333, 0.5])
@pytest.mark.parametrize("side,w", [("R", 0), ("L", 1)])
def test_appB_ev_half_planes(orc, nu, side, w):
    """App. B right/left half-plane stencils == oracle wedge operator (per half)."""
    rng = np.random.default_rng(7)
    for _ in range(5):
        Z = rng.uniform(0.5, 2.0)
        U, Vv, P = rng.normal(size=(3, 3, 3))
        out = orc.wedge_apply(1, w, nu, np.stack([P / Z, U, Vv]))
        A = lambda n: appB(f"{side}_{n}", nu)
        u = (A("uu") * U).sum() + (A("uv") * Vv).sum() + (A("up") * P).sum() / Z
        v = (A("uv") * U).sum() + (A("vv") * Vv).sum() + (A("vp") * P).sum() / Z
        p = Z * (A("up") * U).sum() + Z * (A("vp") * Vv).sum() + (A("pp") * P).sum()
        np.testing.assert_allclose([out[1], out[2], Z * out[0]], [u, v, p], rtol=0, atol=1e-13)


def test_block_constants_preserved(orc):
    """Sum of the q=0 blocks over the wedges of any node is the identity (constants
    are preserved, Sec. 4 'Why the center increment is essential')."""
    for masks in ([1, 2, 4, 8], [9, 6], [3, 12], [15]):
        S = sum(orc.monomial_block(0, 0, m) for m in masks)
        np.testing.assert_allclose(S, np.eye(3), atol=1e-15)


# ---------------------------------------------------------------------------
# Whole-grid increments for smooth/piecewise data (through orc.increments)
# ---------------------------------------------------------------------------

def _state_from_fields(fr, fu, fv, fp, n, gamma=GAMMA):
    """Build a state (h = 1) whose point values sample the given primitive field
    evaluators f(x, y) and whose averages make the recovered centre equal the field
    at the cell centre (tensor Simpson of U at the nine nodes)."""
    s = np.zeros((16, n, n))
    I, J = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float))
    for base, dx, dy in ((4, 0, 0), (8, 0, 0.5), (12, 0.5, 0)):
        for k, f in enumerate((fr, fu, fv, fp)):
            s[base + k] = f(I + dx, J + dy)
    wq = [1 / 6, 4 / 6, 1 / 6]
    for a in range(3):
        for b in range(3):
            X, Y = I + 0.5 * a, J + 0.5 * b
            r, u, v, p = fr(X, Y), fu(X, Y), fv(X, Y), fp(X, Y)
            U = (r, r * u, r * v, p / (gamma - 1) + 0.5 * r * (u * u + v * v))
            for k in range(4):
                s[k] += wq[a] * wq[b] * U[k]
    return s


NODE_POS = {0: (0.0, 0.0), 1: (0.0, 0.5), 2: (0.5, 0.0), 3: (0.5, 0.5)}


def _scaled_poly(rng, amp, base):
    c = amp * rng.uniform(-1, 1, size=(3, 3))
    c[0, 0] = base
    return c


def test_taylor_series_global_q2(orc):
    """For globally Q2 data the node operator at V, Ev, Eh and C equals the exact
    solution (terminating Cauchy-Kowalevskaya series) of the frozen system."""
    n, sc = 10, 5.0
    rng = np.random.default_rng(11)
    cr, cu, cv, cp = (_scaled_poly(rng, 0.1, b) for b in (1.0, 0.3, -0.2, 1.0))
    # polynomial in the scaled variable (x - sc)/sc: still Q2 in (x, y)
    ev = lambda c: (lambda X, Y: qf.poly2d_eval(c, (X - sc) / sc, (Y - sc) / sc))
    s = _state_from_fields(ev(cr), ev(cu), ev(cv), ev(cp), n)
    for tau in (0.05, 0.21, 0.38):
        inc, _ = orc.increments(s, 1.0, GAMMA, tau, threads=1)
        for fam in range(4):
            for j in range(3, n - 3):
                for i in range(3, n - 3):
                    x, y = i + NODE_POS[fam][0], j + NODE_POS[fam][1]
                    X, Y = (x - sc) / sc, (y - sc) / sc
                    rK, uK, vK, pK = (qf.poly2d_eval(c, X, Y) for c in (cr, cu, cv, cp))
                    cK = math.sqrt(GAMMA * pK / rK)
                    ZK = rK * cK
                    assert cK * tau <= 0.5
                    # CK in the scaled variable: derivative factor 1/sc -> speed cK/sc
                    pi, u, v = qf.ck_solution(cp / ZK, cu, cv, cK / sc, tau, X, Y)
                    got = inc[fam, :, j, i]
                    want = [u - uK, v - vK, ZK * pi - pK]
                    np.testing.assert_allclose(got, want, rtol=0, atol=2e-14)


def _kinked_1d(rng, x0, base, amp):
    """Continuous piecewise quadratic in x with a kink at x0."""
    a, bl, br, cl, cr = base, *(amp * rng.uniform(-1, 1, size=4))

    def f(X):
        d = X - x0
        return np.where(d < 0, a + bl * d + cl * d * d, a + br * d + cr * d * d)
    return f


@pytest.mark.parametrize("axis", [0, 1])
def test_dalembert_kink(orc, axis):
    """One-dimensional data with a kink on a grid line: every node (quadrant sums at
    vertices, half-planes at edges, the disk at centres) reproduces d'Alembert."""
    n, x0 = 10, 5.0
    rng = np.random.default_rng(3 + axis)
    fr, fn, ft, fp = (_kinked_1d(rng, x0, b, a) for b, a in ((1.0, 0.05), (0.2, 0.08), (-0.1, 0.08), (1.0, 0.05)))
    pick = (lambda f: (lambda X, Y: f(X))) if axis == 0 else (lambda f: (lambda X, Y: f(Y)))
    # normal velocity follows the kink axis
    if axis == 0:
        s = _state_from_fields(pick(fr), pick(fn), pick(ft), pick(fp), n)
    else:
        s = _state_from_fields(pick(fr), pick(ft), pick(fn), pick(fp), n)
    for tau in (0.13, 0.36):
        inc, _ = orc.increments(s, 1.0, GAMMA, tau, threads=1)
        for fam in range(4):
            for j in range(3, n - 3):
                for i in range(3, n - 3):
                    x, y = i + NODE_POS[fam][0], j + NODE_POS[fam][1]
                    xx = x if axis == 0 else y
                    rK, pK = fr(np.array(xx)), fp(np.array(xx))
                    cK = math.sqrt(GAMMA * pK / rK)
                    ZK = rK * cK
                    d = cK * tau
                    wp = lambda X: fn(np.array(X)) + fp(np.array(X)) / ZK
                    wm = lambda X: fn(np.array(X)) - fp(np.array(X)) / ZK
                    un = 0.5 * (wp(xx - d) + wm(xx + d))
                    pi = 0.5 * (wp(xx - d) - wm(xx + d))
                    dn = un - fn(np.array(xx))
                    dp = ZK * pi - pK
                    got = inc[fam, :, j, i]
                    want = [dn, 0.0, dp] if axis == 0 else [0.0, dn, dp]
                    np.testing.assert_allclose(got, want, rtol=0, atol=2e-14)


# ---------------------------------------------------------------------------
# General 2-D piecewise data: Poisson formula
# ---------------------------------------------------------------------------

# node family -> (position on a 2x2-cell patch with lower-left corner (0,0),
#                 face lines through it, wedge cells in the oracle's wedge order)
PATCH = {
    0: ((1.0, 1.0), (True, True), [(1, 1), (0, 1), (0, 0), (1, 0)]),
    1: ((1.0, 0.5), (True, False), [(1, 0), (0, 0)]),
    2: ((0.5, 1.0), (False, True), [(0, 1), (0, 0)]),
    3: ((0.5, 0.5), (False, False), [(0, 0)]),
}


@pytest.mark.parametrize("fam", [0, 1, 2, 3])
def test_poisson_formula_piecewise(orc, fam):
    rng = np.random.default_rng(100 + fam)
    K, lines, cells = PATCH[fam]
    for trial in range(3):
        npi, nu, nv = rng.normal(size=(3, 5, 5))
        fpi, fu, fv = qf.PiecewiseQ2(npi), qf.PiecewiseQ2(nu), qf.PiecewiseQ2(nv)
        for r in (0.11, 0.3, 0.5):
            got = np.zeros(3)
            for w, (ci, cj) in enumerate(cells):
                f = np.stack([a[2 * ci:2 * ci + 3, 2 * cj:2 * cj + 3] for a in (npi, nu, nv)])
                got += orc.wedge_apply(fam, w, r, f)
            want = qf.poisson_node(fpi, fu, fv, K, lines, 1.0, r)
            np.testing.assert_allclose(got, want, rtol=0, atol=5e-13)
