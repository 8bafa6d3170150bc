"""Pins of the oracle's diagnostics against closed forms (no GPU).

* conservative totals are h^2 times the sums of the averages, which for data given by
  cell averages of a periodic field equal its exact integrals;
* the entropy functional -int rho log(p / rho^gamma) dA, discretised by the tensor
  Simpson rule over the nine Q2 nodes of every cell (the recovered centre included),
  converges at fourth order to the exact integral of a smooth non-isentropic field;
* minima, maxima and the acoustic CFL number over the nodes are the extremes of the
  sampled values.
"""
import math

import numpy as np

from paper_2605_12915_amd import inputs as I

G = 1.4


def field(xv, yv):
    X, Y = np.meshgrid(xv, yv)
    rho = 1.0 + 0.3 * np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y)
    u = 0.2 * np.cos(2 * math.pi * Y)
    v = -0.1 * np.sin(2 * math.pi * X)
    p = 1.0 + 0.2 * np.cos(2 * math.pi * (X + Y))
    return rho, u, v, p


def exact_integrals():
    """Gauss-Legendre tensor quadrature, 64 x 64 panels of 12 x 12 points: exact to
    round-off for these trigonometric integrands."""
    g, w = np.polynomial.legendre.leggauss(12)
    panels = 64
    x = ((np.arange(panels)[:, None] + 0.5 * (g[None, :] + 1.0)) / panels).reshape(-1)
    wx = np.tile(0.5 * w / panels, panels)
    rho, u, v, p = field(x, x)
    W = np.outer(wx, wx)
    E = p / (G - 1.0) + 0.5 * rho * (u * u + v * v)
    return {"mass": float(np.sum(W * rho)), "momx": float(np.sum(W * rho * u)),
            "momy": float(np.sum(W * rho * v)), "energy": float(np.sum(W * E)),
            "entropy": float(-np.sum(W * rho * (np.log(p) - G * np.log(rho))))}


def problem(n):
    return I.Problem("diag_field", n, n, 0.0, 0.0, 1.0 / n, G, field)


def test_totals_are_exact_integrals(orc):
    ex = exact_integrals()
    P = problem(24)
    d = orc.diagnostics(P.state(), P.h, G, 1e-3)
    for k in ("mass", "momx", "momy", "energy"):
        # the 5x5 Gauss-Legendre cell averages integrate these smooth fields to ~1e-12
        assert abs(d[k] - ex[k]) <= 1e-10 * max(1.0, abs(ex[k])), (k, d[k], ex[k])


def test_entropy_fourth_order(orc):
    ex = exact_integrals()["entropy"]
    errs = []
    for n in (8, 16, 32, 64):
        P = problem(n)
        errs.append(abs(orc.diagnostics(P.state(), P.h, G, 1e-3)["entropy"] - ex))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    print("entropy errors", errs, "orders", orders)
    # Simpson error ~ h^4 f^(4) / 180: 6e-9 at n = 64 for this field (|ex| = 0.041)
    assert errs[-1] < 1e-8
    assert min(orders[1:]) > 3.5, orders


def _cons(w):
    r, u, v, p = w
    return np.stack([r, r * u, r * v, p / (G - 1.0) + 0.5 * r * (u * u + v * v)])


def _prim(U):
    r = U[0]
    u, v = U[1] / r, U[2] / r
    return np.stack([r, u, v, (G - 1.0) * (U[3] - 0.5 * r * (u * u + v * v))])


def test_extremes_over_nodes(orc):
    """Minima and maxima over the four node families, with the centre obtained here
    from its defining condition: the 3x3 Simpson average of the Q2 interpolant of the
    conserved variables equals the cell average (corner weight 1/36, edge 4/36,
    centre 16/36)."""
    n = 20
    P = I.Problem("diag_field", n, n, 0.0127, 0.0311, 1.0 / n, G, field)
    s = P.state()
    dt = 2e-3
    d = orc.diagnostics(s, P.h, G, dt)
    UV, UEv, UEh = _cons(s[4:8]), _cons(s[8:12]), _cons(s[12:16])
    sh = lambda a, dx, dy: np.roll(np.roll(a, -dy, axis=1), -dx, axis=2)
    corners = UV + sh(UV, 1, 0) + sh(UV, 0, 1) + sh(UV, 1, 1)
    edges = UEv + sh(UEv, 1, 0) + UEh + sh(UEh, 0, 1)
    C = _prim((36.0 * s[0:4] - corners - 4.0 * edges) / 16.0)
    fams = [s[4:8], s[8:12], s[12:16], C]
    rho = np.concatenate([q[0].ravel() for q in fams])
    p = np.concatenate([q[3].ravel() for q in fams])
    cs = np.sqrt(G * p / rho)
    spd = np.concatenate([np.hypot(q[1], q[2]).ravel() for q in fams]) + cs
    assert np.isclose(d["min_rho"], rho.min(), rtol=1e-13, atol=0)
    assert np.isclose(d["min_p"], p.min(), rtol=1e-13, atol=0)
    assert np.isclose(d["max_speed"], spd.max(), rtol=1e-13, atol=0)
    assert np.isclose(d["max_acoustic_r"], cs.max() * dt / P.h, rtol=1e-13, atol=0)
    # the centres matter: without them the extremes differ for this field
    nn = 3 * n * n
    assert rho[nn:].min() < rho[:nn].min() or spd[nn:].max() > spd[:nn].max()


# Vorticity of the piecewise-Q2 velocity reconstruction.  For `field`:
# omega = dv/dx - du/dy = -0.2 pi cos(2 pi x) + 0.4 pi sin(2 pi y), so over the unit
# square int omega = 0 and int omega^2 = (0.2 pi)^2 / 2 + (0.4 pi)^2 / 2 = 0.1 pi^2.
ENSTROPHY_EXACT = 0.1 * math.pi ** 2


def test_vorticity_integral_vanishes_on_periodic_grids(orc):
    # smooth data, and rough random node values: the reconstruction is continuous, so
    # the cell integrals of its curl telescope to zero whatever the data
    rng = np.random.default_rng(5)
    for s in (problem(24).state(), problem(17).state() + 0.05 * rng.normal(size=(16, 17, 17)) * np.r_[
            np.zeros(4), np.tile([0.0, 1.0, 1.0, 0.0], 3)][:, None, None]):
        d = orc.diagnostics(s, 1.0 / s.shape[2], G, 1e-3)
        assert abs(d["vorticity"]) < 1e-14 * max(1.0, math.sqrt(d["enstrophy"])), d["vorticity"]
        assert d["enstrophy"] > 0.1


def test_enstrophy_converges_to_exact(orc):
    errs = []
    for n in (8, 16, 32, 64):
        P = problem(n)
        errs.append(abs(orc.diagnostics(P.state(), P.h, G, 1e-3)["enstrophy"] - ENSTROPHY_EXACT))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    print("enstrophy errors", errs, "orders", orders)
    assert errs[-1] < 1e-5 * ENSTROPHY_EXACT
    assert min(orders[1:]) > 3.5, orders


def _transpose(s):
    """Swap x and y: averages (rho, rho v, rho u, E), vertices (rho, v, u, p), and the
    two edge families exchange (and swap their velocity components)."""
    t = np.empty_like(s)
    T = lambda a: a.T
    t[0], t[1], t[2], t[3] = T(s[0]), T(s[2]), T(s[1]), T(s[3])
    for dst, src in ((4, 4), (8, 12), (12, 8)):
        t[dst], t[dst + 1], t[dst + 2], t[dst + 3] = T(s[src]), T(s[src + 2]), T(s[src + 1]), T(s[src + 3])
    return t


def test_vorticity_invariances(orc):
    P = problem(20)
    s = P.state()
    d = orc.diagnostics(s, P.h, G, 1e-3)
    # transposition maps omega to -omega
    dt_ = orc.diagnostics(_transpose(s), P.h, G, 1e-3)
    assert abs(dt_["enstrophy"] - d["enstrophy"]) <= 1e-13 * d["enstrophy"]
    # scaling every velocity (point values, and the momentum averages from which the
    # centre's velocity is recovered) scales the enstrophy by the square
    s2 = s.copy()
    s2[1] *= 3.0
    s2[2] *= 3.0
    for b in (4, 8, 12):
        s2[b + 1] *= 3.0
        s2[b + 2] *= 3.0
    assert abs(orc.diagnostics(s2, P.h, G, 1e-3)["enstrophy"] - 9.0 * d["enstrophy"]) <= 1e-12 * d["enstrophy"]
    # a uniform flow has none
    s3 = s.copy()
    for b in (4, 8, 12):
        s3[b + 1] = 0.3
        s3[b + 2] = -0.2
    s3[1] = 0.3 * s3[0]
    s3[2] = -0.2 * s3[0]
    d3 = orc.diagnostics(s3, P.h, G, 1e-3)
    assert abs(d3["enstrophy"]) < 1e-25 and abs(d3["vorticity"]) < 1e-15


def _vel_problem(n, uf, vf):
    def f(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        return 1.0 + 0.0 * X, uf(X, Y), vf(X, Y), 1.0 + 0.0 * X
    return I.Problem("vel_field", n, n, 0.0, 0.0, 1.0 / n, G, f)


def test_enstrophy_sign_sensitive_and_irrotational(orc):
    """u = 0.2 sin(2 pi (x + y)), v = 0.05 sin(2 pi (x + y)): omega = -0.3 pi cos(2 pi (x + y)),
    int omega^2 = 0.045 pi^2 (a sign error between the two curl terms would give
    (0.5 pi)^2 / 2 instead).  A gradient field u = phi_x, v = phi_y has omega = 0."""
    w = lambda X, Y: np.sin(2 * math.pi * (X + Y))
    exact = 0.045 * math.pi ** 2
    e1, e2 = [], []
    for n in (16, 32, 64):
        P = _vel_problem(n, lambda X, Y: 0.2 * w(X, Y), lambda X, Y: 0.05 * w(X, Y))
        e1.append(abs(orc.diagnostics(P.state(), P.h, G, 1e-3)["enstrophy"] - exact))
        # phi = 0.1 sin(2 pi x) sin(2 pi y) / (2 pi)
        Q = _vel_problem(n, lambda X, Y: 0.1 * np.cos(2 * math.pi * X) * np.sin(2 * math.pi * Y),
                         lambda X, Y: 0.1 * np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y))
        e2.append(orc.diagnostics(Q.state(), Q.h, G, 1e-3)["enstrophy"])
    print("sign-sensitive errors", e1, "irrotational enstrophy", e2)
    assert e1[-1] < 1e-5 * exact and math.log2(e1[-2] / e1[-1]) > 3.5
    assert e2[-1] < 1e-6 and math.log2(e2[-2] / e2[-1]) > 3.5


def test_experiment_initial_data():
    """Sec. 6 initial data as stated: the shear's band indicator a(y) is 1 inside
    |y| < 7/32, 0 outside |y| >= 9/32 and continuous (with its slope) at the four
    breakpoints; the Kelvin-Helmholtz layer has rho in [1/2, 2] and u = (B - 1)/2."""
    P = I.low_mach_shear(64)
    assert (P.nx, P.ny, P.x0, P.y0, P.h) == (64, 32, 0.0, -0.5, 2.0 / 64)
    y = np.array([-0.5, -9 / 32 - 1e-12, -9 / 32, -7 / 32 - 1e-12, -7 / 32, 0.0, 7 / 32 - 1e-12, 7 / 32,
                  9 / 32 - 1e-12, 9 / 32, 0.49])
    rho, u, v, p = P.prim(np.array([0.25]), y)
    a = (1.0 - u[:, 0] / 1e-2) / 2.0
    assert np.allclose(a, [0, 0, 0, 1, 1, 1, 1, 1, 0, 0, 0], atol=1e-9)
    assert np.allclose(rho[:, 0], G + 1e-3 * (1.0 - 2.0 * a)) and np.allclose(p, 1.0)
    assert np.allclose(v, 0.1 * 1e-2 * math.sin(2 * math.pi * 0.25))
    Q = I.kelvin_helmholtz(64)
    rho, u, v, p = Q.prim(np.array([-1.0, -0.25, 0.5]), np.array([-1.0, 0.0, 0.9]))
    B = np.tanh(15 * np.array([-1.0, 0.0, 0.9]) + 7.5) - np.tanh(15 * np.array([-1.0, 0.0, 0.9]) - 7.5)
    assert np.allclose(rho, (0.5 + 0.75 * B)[:, None]) and np.allclose(u, (0.5 * (B - 1.0))[:, None])
    assert np.allclose(v, 0.1 * np.sin(2 * math.pi * np.array([-1.0, -0.25, 0.5]))[None, :]) and np.allclose(p, 1.0)
    assert 0.5 - 1e-6 < rho.min() and rho.max() < 2.0
