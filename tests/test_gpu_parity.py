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


@pytest.mark.parametrize("nx,ny,steps", [(4, 4, 5), (5, 7, 4), (37, 29, 6), (70, 9, 3), (9, 70, 3), (31, 10, 4),
                                         (62, 20, 4), (12, 200, 2), (200, 12, 2)])
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


def _converging(n=32):
    """Uniform rho = p = 1 with u = -0.5 sin(2 pi x): the compression near x = 0 heats
    the gas, so that at acoustic CFL 0.494 (0.496) of the initial sound speed the
    guard c dt / h <= 1/2 holds for two (one) steps and fires at the third (second)."""
    def prim(xv, yv):
        X, Y = np.meshgrid(xv, yv)
        return (np.ones_like(X), -0.5 * np.sin(2 * math.pi * X), np.zeros_like(X), np.ones_like(X))
    return I.Problem("converging", n, n, 0.0, 0.0, 1.0 / n, 1.4, prim, bg=(1.0, 0.0, 0.0, 1.0))


def _oracle_statuses(orc, P, s0, dt, n):
    x, out = s0, []
    for _ in range(n):
        r = orc.step(x, P.h, P.gamma, dt, check=False)
        if isinstance(r, tuple):
            x, st = r
        else:
            x, st = r, 0
        out.append(st)
    return out


def test_foot_status(torch_dev, orc):
    """A supersonic state (u = 3, p = 0.01, c = 0.12) at dt = 0.4 h moves every foot 1.2
    cells: AF_ERR_FOOT (the kernel clamps the feet to their nodes, so every gather stays
    in the halo and the launch ends normally) and the input is returned unchanged."""
    torch, dev = torch_dev
    from paper_2605_12915_amd._lib import AF_ERR_FOOT, AfError
    from paper_2605_12915_amd.stepper import Stepper
    P = I.uniform(12, W=(1.0, 3.0, 0.0, 0.01), ny=10)
    s0 = P.state()
    dt = 0.4 * P.h
    assert _oracle_statuses(orc, P, s0, dt, 1) == [2]           # the oracle's foot status
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev, check_errors=True)
    for n in (1, 3):
        print("foot status, nsteps", n, flush=True)
        x = torch.from_numpy(s0).to(dev)
        with pytest.raises(AfError) as e:
            st.step(x, dt, n)
        assert e.value.code == AF_ERR_FOOT
        assert np.array_equal(x.cpu().numpy(), s0)
    # without AF_CHECK the bit accumulates on the device and af_read_status reports it
    st2 = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    x = torch.from_numpy(s0).to(dev)
    st2.step(x, dt, 1)
    assert st2.read_status() == AF_ERR_FOOT
    assert st2.read_status() == 0


@pytest.mark.parametrize("r0,nsteps,fails_at", [(0.494, 3, 2), (0.496, 2, 1)])
def test_check_rolls_back_to_input(torch_dev, orc, r0, nsteps, fails_at):
    """AF_CHECK with a check that fires after some steps succeeded: the call returns the
    status and *inout holds the input of the call (not the last good step)."""
    torch, dev = torch_dev
    from paper_2605_12915_amd._lib import AF_ERR_ACOUSTIC_CFL, AfError
    from paper_2605_12915_amd.stepper import Stepper
    P = _converging()
    s0 = P.state()
    dt = r0 * P.h / math.sqrt(1.4)
    sts = _oracle_statuses(orc, P, s0, dt, nsteps)
    assert sts[:fails_at] == [0] * fails_at and sts[fails_at] == 1, sts
    print("rollback case", r0, nsteps, sts, flush=True)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev, check_errors=True)
    x = torch.from_numpy(s0).to(dev)
    with pytest.raises(AfError) as e:
        st.step(x, dt, nsteps)
    assert e.value.code == AF_ERR_ACOUSTIC_CFL
    assert np.array_equal(x.cpu().numpy(), s0)
    # the steps before the failing one are fine: stepping them alone matches the oracle
    # (the v planes are zero up to round-off here: absolute error for them)
    st.step(x, dt, fails_at)
    got, want = x.cpu().numpy(), orc.run(s0, P.h, P.gamma, dt, fails_at)
    scale = np.maximum(np.abs(want).max(axis=(1, 2)), 1.0)
    assert (np.abs(got - want).max(axis=(1, 2)) / scale).max() <= TOL


@pytest.mark.parametrize("vel", [(1.9, -1.7), (1.5, -1.45)])
def test_general_foot_branch(torch_dev, orc, vel):
    """Near Mach 2 at dt = 0.4 h / c the half-step and full-step first-stage feet of
    edge-midpoint targets lie on different sides of the neighbouring face, so those
    targets leave the shared-cell path of the paired point update and take the general
    two-stage path (all of them at (1.9, -1.7); a mix of both paths within the same
    wavefronts at (1.5, -1.45)).  Against the oracle to the FP64 bar."""
    P = I.random_smooth(40, 36, seed=21, amp=0.08, vel=vel)
    s0 = P.state()
    dt = 0.4 * P.h / math.sqrt(1.4)
    lam1 = dt / P.h
    u_eh = s0[13]
    straddle = np.floor(0.5 - 0.5 * lam1 * u_eh) != np.floor(0.5 - lam1 * u_eh)
    print("general foot branch", vel, "EH targets straddling:", straddle.mean(), flush=True)
    assert straddle.mean() > 0.5
    want = orc.run(s0, P.h, P.gamma, dt, 3)
    got, _ = _run_gpu(torch_dev, P, s0, dt, 3, check_errors=True)
    assert _err(got, want).max() <= TOL


def test_run_twice_bitwise(torch_dev):
    """The forward step has no atomics in its arithmetic (only the status OR): two runs
    of the same steps give the same bits, FP64 and FP32."""
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper, to_perturbation
    P = I.fourier_modes(512)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    outs = []
    for prec in ("f64", "f32"):
        for rep in range(2):
            st = Stepper(P.nx, P.ny, P.h, P.gamma, precision=prec, bg=P.bg, device=dev)
            x = torch.from_numpy(s0 if prec == "f64" else to_perturbation(s0, P.bg, P.gamma)).to(dev)
            st.step(x, dt, 10)
            torch.cuda.synchronize()
            outs.append(x.cpu().numpy())
            st.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[2], outs[3])


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


def test_fourier_modes_2048_20_steps(torch_dev, orc):
    """The benchmark's 2048^2 flow over 20 steps (its launch configuration), every
    output against the oracle run on the host cores."""
    P = I.fourier_modes(2048)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    print("2048^2 Fourier-mode flow: oracle 20 steps ...", flush=True)
    want = orc.run(s0, P.h, P.gamma, dt, 20)
    got, _ = _run_gpu(torch_dev, P, s0, dt, 20, check_errors=True)
    err = _err(got, want)
    print("2048^2 20 steps per-plane error", err.max(), flush=True)
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
