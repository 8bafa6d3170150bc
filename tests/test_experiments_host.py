"""Host logic of the experiment drivers (paper_2605_12915_amd/experiments.py): the
radial-asymmetry measure of the acoustic pulse."""
import numpy as np

from paper_2605_12915_amd import experiments as E
from paper_2605_12915_amd import inputs as I


def _state_of(f, n, L=8.0):
    """Point planes of the pressure field f(x, y) on the [-L/2, L/2]^2 grid."""
    h = L / n
    x = -L / 2 + h * np.arange(n)
    s = np.zeros((16, n, n))
    s[7] = f(x[None, :], x[:, None])
    s[11] = f(x[None, :], x[:, None] + h / 2)
    s[15] = f(x[None, :] + h / 2, x[:, None])
    return s


def test_radial_field_has_no_asymmetry():
    s = I.paper_pulse(80).state()
    assert E.radial_asymmetry(s, 80) < 1e-14
    assert E.radial_asymmetry(_state_of(lambda x, y: np.cos(x * x + y * y), 64), 64) < 1e-14


def test_direction_dependence_detected():
    # invariant under the grid's symmetries but not radial: x^4 + y^4 differs from
    # (x^2 + y^2)^2 / 2 along the diagonal, e.g. nodes (5, 0) and (3, 4) cells
    n, h = 64, 8.0 / 64
    a = E.radial_asymmetry(_state_of(lambda x, y: x ** 4 + y ** 4, n), n)
    r4 = (5 * h) ** 4
    assert a >= r4 - ((3 * h) ** 4 + (4 * h) ** 4) - 1e-12
    # one perturbed node
    s = I.paper_pulse(80).state()
    s[11, 30, 47] += 3e-4
    assert abs(E.radial_asymmetry(s, 80) - 3e-4) < 1e-12
