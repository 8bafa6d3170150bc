"""Pins of the foot-centred exact frozen-acoustic update (oracle/footcentred.py; App. C
and the paragraph of Sec. 4 on an exact frozen acoustic update).

The off-centre acoustic operator is pinned where the exact solution is known by
other means:
  * global Q2 polynomial data: the terminating Cauchy-Kowalevskaya series
    (tests/q2field.ck_solution), at feet inside a cell, near a face, near a corner,
    on a node, for radii up to 0.45 cells;
  * data varying in one direction with kinks at the grid lines: d'Alembert's
    formula, which exercises the line terms of the distributional gradient and the
    caps; data varying in x plus data varying in y (both lines and the double cap);
  * a disk centred on a node: the Poisson-formula helper tests/q2field.poisson_node
    and the node-centred operator of the C++ oracle (App. D blocks).
The history term of the velocity is pinned against the form App. C writes (radius
integral of spherical means plus chord terms for the jumps of div u).  The step built
on it is pinned by free-stream preservation, discrete conservation, and the fluid at
rest, where the foot is the node and the update must equal the transported
(node-centred) update of the C++ oracle.
"""
import math

import numpy as np
import pytest

from oracle import footcentred as fc
from paper_2605_12915_amd import inputs as I

from tests import q2field as q


def lattice_of(fun, nx=8, ny=8):
    L = np.zeros((2 * nx, 2 * ny))
    for a in range(2 * nx):
        for b in range(2 * ny):
            L[a, b] = fun(a / 2.0, b / 2.0)
    return fc.Q2Lattice(L)


FEET = [(3.3, 4.2), (3.0, 4.0), (3.9, 4.05), (3.5, 4.5), (3.02, 3.97), (4.0, 3.61), (3.45, 5.0)]
RADII = [0.05, 0.2, 0.45]


@pytest.mark.parametrize("seed", [1, 2])
def test_global_polynomial_equals_ck_series(seed):
    rng = np.random.default_rng(seed)
    cp, cu, cv = (rng.normal(size=(3, 3)) for _ in range(3))
    fp = lattice_of(lambda x, y: q.poly2d_eval(cp, x, y))
    fu = lattice_of(lambda x, y: q.poly2d_eval(cu, x, y))
    fv = lattice_of(lambda x, y: q.poly2d_eval(cv, x, y))
    for F in FEET:
        for R in RADII:
            got = fc.exact_acoustic(F, R, fp, fu, fv)
            want = np.array(q.ck_solution(cp, cu, cv, 1.0, R, F[0], F[1]))
            scale = max(1.0, np.abs(want).max())
            assert np.abs(got - want).max() <= 2e-13 * scale, (F, R, got, want)


def _kinked_1d(seed, n=16):
    """A continuous piecewise-quadratic function on the half-integer lattice (random
    nodal values), evaluated exactly by the same Lagrange basis."""
    vals = np.random.default_rng(seed).normal(size=2 * n + 1)

    def f(x):
        x = np.asarray(x, float)
        c = np.floor(x).astype(int)
        s = 2.0 * (x - c) - 1.0
        L = [0.5 * s * (s - 1.0), 1.0 - s * s, 0.5 * s * (s + 1.0)]
        return sum(L[a] * vals[(2 * c + a) % (2 * n)] for a in range(3))

    return f


def test_one_dimensional_kinks_equal_dalembert():
    """pi_0(x), u_0(x) continuous piecewise quadratics with kinks at integer x, v_0 = 0:
    the 2-D solution is d'Alembert's, (u + pi)(x - R) and (u - pi)(x + R)."""
    p0, u0 = _kinked_1d(3), _kinked_1d(4)
    fp = lattice_of(lambda x, y: p0(x))
    fu = lattice_of(lambda x, y: u0(x))
    fv = lattice_of(lambda x, y: 0.0)
    for F in FEET:
        for R in RADII:
            x = F[0]
            a, b = u0(x - R) + p0(x - R), u0(x + R) - p0(x + R)
            want = np.array([0.5 * (a - b), 0.5 * (a + b), 0.0])
            got = fc.exact_acoustic(F, R, fp, fu, fv)
            assert np.abs(got - want).max() <= 2e-13, (F, R, got, want)
    # the same along y
    fp = lattice_of(lambda x, y: p0(y))
    fu = lattice_of(lambda x, y: 0.0)
    fv = lattice_of(lambda x, y: u0(y))
    for F in FEET:
        R = 0.37
        y = F[1]
        a, b = u0(y - R) + p0(y - R), u0(y + R) - p0(y + R)
        want = np.array([0.5 * (a - b), 0.0, 0.5 * (a + b)])
        assert np.abs(fc.exact_acoustic(F, R, fp, fu, fv) - want).max() <= 2e-13


def test_kinks_in_both_directions_superpose():
    """pi_0 = p1(x) + p2(y), u_0 = u1(x), v_0 = v2(y): the solution is the sum of the two
    one-dimensional solutions; near a corner the disk is cut by both lines (caps and
    the double cap)."""
    p1, p2, u1, v2 = (_kinked_1d(s) for s in (5, 6, 7, 8))
    fp = lattice_of(lambda x, y: p1(x) + p2(y))
    fu = lattice_of(lambda x, y: u1(x))
    fv = lattice_of(lambda x, y: v2(y))
    for F in [(3.02, 3.97), (4.1, 3.9), (3.8, 4.3), (3.0, 4.0), (3.5, 4.0)]:
        for R in [0.15, 0.3, 0.45]:
            x, y = F
            ax, bx = u1(x - R) + p1(x - R), u1(x + R) - p1(x + R)
            ay, by = v2(y - R) + p2(y - R), v2(y + R) - p2(y + R)
            want = np.array([0.5 * (ax - bx) + 0.5 * (ay - by), 0.5 * (ax + bx), 0.5 * (ay + by)])
            got = fc.exact_acoustic(F, R, fp, fu, fv)
            assert np.abs(got - want).max() <= 3e-13, (F, R, got, want)


def test_node_centred_disk_equals_poisson_helper():
    """Disk centred on a vertex, an edge midpoint and a cell centre of general
    continuous piecewise-Q2 data: the independent Poisson-formula helper."""
    rng = np.random.default_rng(9)
    nodes = [rng.normal(size=(17, 17)) for _ in range(3)]
    fq = [q.PiecewiseQ2(n) for n in nodes]
    fl = [fc.Q2Lattice(n[:16, :16]) for n in nodes]
    for K, lines in [((4.0, 4.0), (True, True)), ((4.0, 4.5), (True, False)), ((4.5, 4.0), (False, True)),
                     ((4.5, 4.5), (False, False))]:
        for R in (0.2, 0.45):
            want = q.poisson_node(fq[0], fq[1], fq[2], K, lines, 1.0, R)
            got = fc.exact_acoustic(K, R, fl[0], fl[1], fl[2])
            assert np.abs(got - want).max() <= 1e-11 * max(1.0, np.abs(want).max()), (K, R, got, want)


def _history_parts(F, R, fu, fv):
    X, Y, zx, zy, w = fc.disk_nodes(F, R)
    g = fu.eval(X, Y, (1, 0)) + fv.eval(X, Y, (0, 1))
    z2 = zx * zx + zy * zy
    return np.array([R * np.sum(w * g * zx / z2), R * np.sum(w * g * zy / z2)])


def test_history_forms_agree(monkeypatch):
    """The history term of the velocity, int_0^R r M_r[grad g] dr: the disk form that
    exact_acoustic uses (exchange of the integration order, then integration by parts)
    equals the form written in App. C (spherical means of grad g at Gauss radii plus
    the chord integrals of the jumps of g = div u_0 across grid lines), here at raised
    quadrature orders, for general continuous piecewise-Q2 data (random nodal values)
    with grid lines and a corner close to the foot.  The disk form is converged at the
    default orders (unchanged to 1e-15 when they are raised)."""
    rng = np.random.default_rng(12)
    fu, fv = (fc.Q2Lattice(rng.normal(size=(16, 16))) for _ in range(2))
    cases = [((3.02, 3.97), 0.45), ((3.9, 4.05), 0.45), ((3.1, 3.05), 0.3), ((3.3, 4.2), 0.45)]
    default = [_history_parts(F, R, fu, fv) for F, R in cases]
    monkeypatch.setattr(fc, "NQ_THETA", 64)
    monkeypatch.setattr(fc, "NQ_RHO", 20)
    monkeypatch.setattr(fc, "NQ_R", 24)
    monkeypatch.setattr(fc, "_GL", {})
    for (F, R), d in zip(cases, default):
        parts = _history_parts(F, R, fu, fv)
        radius = fc.history_by_radius(F, R, fu, fv)
        scale = max(1.0, np.abs(parts).max())
        assert np.abs(parts - d).max() <= 1e-14 * scale, (F, R, parts, d)
        assert np.abs(parts - radius).max() <= 1e-10 * scale, (F, R, parts, radius)


def test_fluid_at_rest_equals_transported_update(orc):
    """At rest the foot is the node, the frozen state is the node's and the exact
    acoustic update centred there is the node-centred one: the foot-centred point
    values equal the transported update of the C++ oracle, and so does the step."""
    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        g = 0.05 * np.exp(-((X - 0.45) ** 2 + (Y - 0.55) ** 2) / 0.04)
        return 1.0 + g, 0.0 * X, 0.0 * X, 1.0 / 1.4 + g
    P = I.Problem("rest", 5, 5, 0.0, 0.0, 1.0 / 5, 1.4, prim)
    s0 = P.state()
    dt = 0.4 * P.h / 1.05
    for tau in (0.5 * dt, dt):
        got = fc.point_values(s0, P.h, P.gamma, tau)
        _, want, st = orc.feet(s0, P.h, P.gamma, tau)
        assert st == 0
        want = want.reshape(12, *want.shape[2:])
        assert np.abs(got - want).max() <= 1e-13, np.abs(got - want).max()
    got = fc.step(s0, P.h, P.gamma, dt)
    want = orc.step(s0, P.h, P.gamma, dt)
    assert np.abs(got - want).max() <= 1e-13


def test_step_free_stream_and_conservation():
    P = I.uniform(4, W=(1.2, 0.15, -0.1, 0.9))
    s0 = P.state()
    dt = P.dt_for_cfl(0.3)
    got = fc.step(s0, P.h, P.gamma, dt)
    assert np.abs(got - s0).max() <= 1e-14 * np.abs(s0).max()
    P = I.random_smooth(4, 5, seed=3, amp=0.08, vel=(0.2, -0.15))
    s0 = P.state()
    got = fc.step(s0, P.h, P.gamma, P.dt_for_cfl(0.3))
    for k in range(4):
        assert abs(got[k].sum() - s0[k].sum()) <= 1e-14 * np.abs(s0[k]).sum()


def test_moving_flow_close_to_transported_update(orc):
    """A smooth moving flow: the foot-centred and the transported updates approximate
    the same frozen evolution, so one step differs by far less than the step's change
    of the state (both are third-order accurate)."""
    P = I.random_smooth(5, 5, seed=4, amp=0.05, vel=(0.25, 0.15), kmax=1)
    s0 = P.state()
    dt = P.dt_for_cfl(0.3)
    a = fc.step(s0, P.h, P.gamma, dt)
    b = orc.step(s0, P.h, P.gamma, dt)
    change = np.abs(b - s0).max()
    assert np.abs(a - b).max() <= 0.05 * change, (np.abs(a - b).max(), change)


def test_footprint_condition():
    """|delta| + R >= h/2 (total CFL beyond 1/2) is refused."""
    P = I.uniform(4, W=(1.0, 0.2, 0.0, 1.0))
    s0 = P.state()
    with pytest.raises(fc.FootprintError):
        fc.point_values(s0, P.h, P.gamma, 0.5 * P.h / (math.sqrt(1.4) + 0.2) * 1.05)
