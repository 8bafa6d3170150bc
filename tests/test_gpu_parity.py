"""GPU parity of the FP64 HIP step (through the C ABI) against the CPU oracle.

Bar: normwise-relative error per plane max|gpu - oracle| / max|oracle| <= 1e-12
(FP64 path; the oracle and the kernels differ only in rounding order and FMA
contraction)."""
import math

import numpy as np
import pytest

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


def _run_gpu(torch_dev, P, s0, dt, n, **kw):
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev, **kw)
    x = torch.from_numpy(s0).to(dev)
    st.step(x, dt, n)
    torch.cuda.synchronize()
    return x.cpu().numpy(), st


def test_vortex_64_100_steps(torch_dev, orc):
    """Isentropic vortex on [0,10]^2, 64^2, mean flow (1,1), CFL 0.3, 100 steps."""
    P = I.isentropic_vortex(64, uinf=(1.0, 1.0))
    s0 = P.state()
    dt = P.dt_for_cfl(0.3)
    print("64x64 vortex, dt", dt, flush=True)
    want = orc.run(s0, P.h, P.gamma, dt, 100)
    got, _ = _run_gpu(torch_dev, P, s0, dt, 100, check_errors=True)
    err = _err(got, want)
    print("per-plane error", err.max())
    assert err.max() <= TOL, err


@pytest.mark.parametrize("nx,ny,steps", [(4, 4, 5), (5, 7, 4), (37, 29, 6), (70, 9, 3)])
def test_ragged_and_small_grids(torch_dev, orc, nx, ny, steps):
    P = I.random_smooth(nx, ny, seed=nx * 100 + ny, amp=0.1, vel=(0.35, -0.25))
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    print("ragged", nx, ny, flush=True)
    want = orc.run(s0, P.h, P.gamma, dt, steps)
    got, _ = _run_gpu(torch_dev, P, s0, dt, steps, check_errors=True)
    assert _err(got, want).max() <= TOL


def test_rb_scheme(torch_dev, orc):
    P = I.random_smooth(24, 20, seed=9, amp=0.1, vel=(0.3, 0.2))
    s0 = P.state()
    dt = P.dt_for_cfl(0.15)
    want = orc.run(s0, P.h, P.gamma, dt, 5, scheme=1)
    got, _ = _run_gpu(torch_dev, P, s0, dt, 5, scheme="rb")
    assert _err(got, want).max() <= TOL


def test_step_out_leaves_input(torch_dev, orc):
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    P = I.gaussian_pulse(32, amp=0.1, width=0.1)
    s0 = P.state()
    dt = P.dt_for_cfl(0.45)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    x = torch.from_numpy(s0).to(dev)
    y = st.step_out(x, dt)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), s0)
    assert _err(y.cpu().numpy(), orc.step(s0, P.h, P.gamma, dt)).max() <= TOL
    # an output that aliases an input is refused before anything runs
    from paper_2605_12915_amd._lib import AF_ERR_ARG, AfError
    with pytest.raises(AfError) as e:
        st.step_out(x, dt, x)
    assert e.value.code == AF_ERR_ARG
    lam = torch.ones_like(x)
    with pytest.raises(AfError) as e:
        st.adjoint(x, lam, dt, out=lam)
    assert e.value.code == AF_ERR_ARG
    with pytest.raises(AfError) as e:
        st.adjoint(x, lam, dt, out=x)
    assert e.value.code == AF_ERR_ARG
    assert np.array_equal(x.cpu().numpy(), s0)


def test_free_stream(torch_dev):
    P = I.uniform(16, W=(1.3, 0.7, -0.4, 0.9), ny=12)
    s0 = P.state()
    got, _ = _run_gpu(torch_dev, P, s0, P.dt_for_cfl(0.45), 100)
    assert np.max(np.abs(got - s0) / np.abs(s0).max(axis=(1, 2), keepdims=True)) <= 1e-14


def test_conservation_gpu(torch_dev):
    P = I.random_smooth(48, 40, seed=2, amp=0.2)
    s0 = P.state()
    got, _ = _run_gpu(torch_dev, P, s0, P.dt_for_cfl(0.4), 50)
    for k in range(4):
        assert abs(got[k].sum() - s0[k].sum()) <= 1e-13 * np.abs(s0[k]).sum()


def test_error_statuses(torch_dev):
    torch, dev = torch_dev
    from paper_2605_12915_amd._lib import AF_ERR_ACOUSTIC_CFL, AF_ERR_NONPHYSICAL, AfError
    from paper_2605_12915_amd.stepper import Stepper
    P = I.uniform(8, W=(1.0, 0.1, 0.0, 1.0))
    s0 = P.state()
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev, check_errors=True)
    x = torch.from_numpy(s0).to(dev)
    with pytest.raises(AfError) as e:
        st.step(x, 0.51 * P.h / math.sqrt(1.4), 2)
    assert e.value.code == AF_ERR_ACOUSTIC_CFL
    assert np.array_equal(x.cpu().numpy(), s0)
    bad = s0.copy()
    bad[7, 2, 3] = -1.0
    x = torch.from_numpy(bad).to(dev)
    with pytest.raises(AfError) as e:
        st.step(x, 0.1 * P.h, 1)
    assert e.value.code == AF_ERR_NONPHYSICAL
    assert np.array_equal(x.cpu().numpy(), bad)


def test_diagnostics_match_oracle(torch_dev, orc):
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    P = I.isentropic_vortex(40, uinf=(1.0, 1.0))
    s0 = P.state()
    dt = P.dt_for_cfl(0.3)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    got = st.diagnostics(torch.from_numpy(s0).to(dev), dt)
    want = orc.diagnostics(s0, P.h, P.gamma, dt)
    for k, v in want.items():
        assert abs(got[k] - v) <= 1e-12 * max(1.0, abs(v)), (k, got[k], v)


def test_fourier_modes_2048_one_step(torch_dev, orc):
    """2048^2 Fourier-mode flow at CFL 0.4: every output of one step against the
    oracle (the oracle runs the full grid on the host cores)."""
    P = I.fourier_modes(2048)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    print("2048^2 Fourier-mode flow: generating done, oracle step ...", flush=True)
    want = orc.step(s0, P.h, P.gamma, dt)
    got, _ = _run_gpu(torch_dev, P, s0, dt, 1, check_errors=True)
    err = _err(got, want)
    print("2048^2 per-plane error", err.max(), flush=True)
    assert err.max() <= TOL


@pytest.mark.parametrize("variant", ["multi", "split"])
def test_other_variants(torch_dev, orc, monkeypatch, variant):
    """The four-kernel path and the two-launch split path against the oracle too."""
    monkeypatch.setenv("AF_VARIANT", variant)
    P = I.random_smooth(40, 24, seed=12, amp=0.1, vel=(0.3, -0.3))
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    want = orc.run(s0, P.h, P.gamma, dt, 4)
    got, st = _run_gpu(torch_dev, P, s0, dt, 4)
    assert _err(got, want).max() <= TOL
    P = I.random_smooth(5, 70, seed=3, amp=0.1, vel=(-0.3, 0.3))
    s0 = P.state()
    want = orc.run(s0, P.h, P.gamma, dt, 3)
    got, st = _run_gpu(torch_dev, P, s0, dt, 3)
    assert _err(got, want).max() <= TOL


def test_timing_api(torch_dev):
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    P = I.random_smooth(64, 64, seed=1, amp=0.05)
    s0 = P.state()
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    x = torch.from_numpy(s0).to(dev)
    tot, ker = st.time_steps(x, P.dt_for_cfl(0.4), 4)
    assert tot > 0 and 0 < ker <= tot
    assert np.array_equal(x.cpu().numpy(), s0)
