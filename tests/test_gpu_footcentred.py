"""GPU foot-centred exact point update (AF_SCHEME_FC; App. C) through the C ABI against
the oracle's foot-centred step (oracle/footcentred.py).

Bar: per plane max|gpu - oracle| / max|oracle| <= 1e-12 (both evaluate the spherical
means by converged quadratures split along the grid lines; they differ by rounding)."""
import math

import numpy as np
import pytest

from oracle import footcentred as fc
from paper_2605_12915_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def _err(got, want):
    return np.abs(got - want).max(axis=(1, 2)) / np.maximum(np.abs(want).max(axis=(1, 2)), 1e-300)


def _gpu(torch_dev, P, s0, dt, n, scheme="fc", **kw):
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme=scheme, device=dev, **kw)
    x = torch.from_numpy(s0).to(dev)
    st.step(x, dt, n)
    torch.cuda.synchronize()
    out = x.cpu().numpy()
    st.close()
    return out


@pytest.mark.parametrize("nx,ny,seed,vel,kmax,steps", [(10, 8, 3, (0.25, -0.15), 3, 1),
                                                        (9, 11, 5, (-0.3, 0.2), 2, 1),
                                                        (8, 8, 7, (0.2, 0.3), 1, 2)])
def test_fc_step_equals_oracle(torch_dev, nx, ny, seed, vel, kmax, steps):
    P = I.random_smooth(nx, ny, seed=seed, amp=0.08, vel=vel, kmax=kmax)
    s0 = P.state()
    dt = P.dt_for_cfl(0.3)
    print("fc step vs oracle", nx, ny, steps, flush=True)
    got = _gpu(torch_dev, P, s0, dt, steps, check_errors=True)
    want = fc.run(s0, P.h, P.gamma, dt, steps)
    err = _err(got, want)
    print("per-plane error", np.array2string(err, precision=2))
    assert err.max() <= TOL


def test_fc_at_rest_equals_transported(torch_dev):
    """At rest the foot is the node and the disk is node-centred: the foot-centred and the
    transported (node-centred) updates coincide."""
    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        g = 0.05 * np.exp(-((X - 0.45) ** 2 + (Y - 0.55) ** 2) / 0.04)
        return 1.0 + g, 0.0 * X, 0.0 * X, 1.0 / 1.4 + g
    P = I.Problem("rest", 12, 10, 0.0, 0.0, 1.0 / 12, 1.4, prim)
    s0 = P.state()
    dt = 0.4 * P.h / 1.05
    a = _gpu(torch_dev, P, s0, dt, 1)
    b = _gpu(torch_dev, P, s0, dt, 1, scheme="tai")
    assert _err(a, b).max() <= 1e-13


def test_fc_free_stream_and_conservation(torch_dev):
    P = I.uniform(12, W=(1.2, 0.15, -0.1, 0.9))
    s0 = P.state()
    got = _gpu(torch_dev, P, s0, P.dt_for_cfl(0.3), 3)
    assert np.abs(got - s0).max() <= 1e-14 * np.abs(s0).max()
    P = I.random_smooth(16, 12, seed=3, amp=0.08, vel=(0.2, -0.15))
    s0 = P.state()
    got = _gpu(torch_dev, P, s0, P.dt_for_cfl(0.3), 2)
    for k in range(4):
        assert abs(got[k].sum() - s0[k].sum()) <= 1e-14 * np.abs(s0[k]).sum()


def test_fc_footprint_status(torch_dev):
    """|delta| + R >= h/2: AF_ERR_FOOTPRINT, the state returned unchanged (AF_CHECK)."""
    torch, dev = torch_dev
    from paper_2605_12915_amd._lib import AF_ERR_FOOTPRINT, AfError
    from paper_2605_12915_amd.stepper import Stepper
    P = I.uniform(8, W=(1.0, 0.3, 0.0, 1.0))
    s0 = P.state()
    dt = 0.45 * P.h / math.sqrt(1.4)
    with pytest.raises(fc.FootprintError):
        fc.point_values(s0, P.h, P.gamma, dt)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme="fc", device=dev, check_errors=True)
    x = torch.from_numpy(s0).to(dev)
    with pytest.raises(AfError) as e:
        st.step(x, dt, 1)
    assert e.value.code == AF_ERR_FOOTPRINT
    assert np.array_equal(x.cpu().numpy(), s0)


def test_fc_unsupported_combinations(torch_dev):
    torch, dev = torch_dev
    from paper_2605_12915_amd._lib import AF_ERR_ARG, AF_ERR_UNSUPPORTED, AfError
    from paper_2605_12915_amd.stepper import Stepper
    P = I.uniform(8, W=(1.0, 0.3, 0.0, 1.0))
    with pytest.raises(AfError) as e:
        Stepper(P.nx, P.ny, P.h, P.gamma, precision="f32", bg=(1.0, 0.3, 0.0, 1.0), scheme="fc", device=dev)
    assert e.value.code == AF_ERR_UNSUPPORTED
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme="fc", device=dev)
    x = torch.from_numpy(P.state()).to(dev)
    with pytest.raises(AfError) as e:
        st.adjoint(x, x.clone(), P.dt_for_cfl(0.3))
    assert e.value.code == AF_ERR_UNSUPPORTED
    assert st.dominant_kernel() == "af::k_fc_points"


def test_fc_benchmark_size_sampled(torch_dev):
    """The benchmark's 256^2 Fourier-mode flow at CFL 0.4, one step: the new point values
    of 30 random targets against the oracle's, target by target, and the averages of 6
    random cells against the oracle's update from the oracle's half- and full-step values
    of the eight targets each cell's edge fluxes use."""
    P = I.fourier_modes(256)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    got = _gpu(torch_dev, P, s0, dt, 1, check_errors=True)
    n = P.nx
    rng = np.random.default_rng(17)
    targets = [(int(f), int(i), int(j)) for f, i, j in zip(rng.integers(0, 3, 30), rng.integers(0, n, 30),
                                                           rng.integers(0, n, 30))]
    want = fc.point_values_at(s0, P.h, P.gamma, dt, targets)
    for (f, i, j), w in zip(targets, want):
        g = got[4 + 4 * f:8 + 4 * f, j, i]
        assert np.abs(g - w).max() <= TOL * max(1.0, np.abs(w).max()), ((f, i, j), g, w)
    # averages of sampled cells (periodic neighbours)
    gam = P.gamma
    cells = [(int(i), int(j)) for i, j in zip(rng.integers(0, n, 6), rng.integers(0, n, 6))]
    for i, j in cells:
        ip, jp = (i + 1) % n, (j + 1) % n
        need = [(0, i, j), (0, ip, j), (0, i, jp), (0, ip, jp), (1, i, j), (1, ip, j), (2, i, j), (2, i, jp)]
        half = fc.point_values_at(s0, P.h, gam, 0.5 * dt, need)
        full = fc.point_values_at(s0, P.h, gam, dt, need)
        now = np.array([s0[4 + 4 * f:8 + 4 * f, b, a] for f, a, b in need])
        tf = lambda fl, k: (fl(now[k], gam) + 4.0 * fl(half[k], gam) + fl(full[k], gam)) / 6.0
        FV = {k: tf(fc._flux_x, k) for k in range(4)}
        GV = {k: tf(fc._flux_y, k) for k in range(4)}
        FE = {k: tf(fc._flux_x, k) for k in (4, 5)}
        GE = {k: tf(fc._flux_y, k) for k in (6, 7)}
        Fl = (FV[0] + 4.0 * FE[4] + FV[2]) / 6.0
        Fr = (FV[1] + 4.0 * FE[5] + FV[3]) / 6.0
        Gb = (GV[0] + 4.0 * GE[6] + GV[1]) / 6.0
        Gt = (GV[2] + 4.0 * GE[7] + GV[3]) / 6.0
        want_avg = s0[0:4, j, i] - dt / P.h * ((Fr - Fl) + (Gt - Gb))
        g = got[0:4, j, i]
        assert np.abs(g - want_avg).max() <= TOL * np.abs(want_avg).max(), ((i, j), g, want_avg)

