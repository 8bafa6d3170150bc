"""FP64 adjoint step (af_step_adjoint) against the oracle.

* exact parity: on a small grid the oracle's full Jacobian is assembled column by
  column from complex-step JVPs (exact to round-off) and J^T lambda compared with
  the GPU adjoint element by element;
* dot-product test on a larger grid: <lambda, J v> (oracle JVP) = <J^T lambda, v> (GPU);
* checkpointed rollout gradient against central finite differences (GPU forward).
"""

import numpy as np
import pytest

from paper_2605_12915_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def gpu_adjoint(torch_dev, P, s0, lam, dt, scheme="tai"):
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme=scheme, device=dev)
    g = st.adjoint(torch.from_numpy(s0).to(dev), torch.from_numpy(np.ascontiguousarray(lam)).to(dev), dt)
    torch.cuda.synchronize()
    return g.cpu().numpy()


# tiny grids (windows wrapping onto themselves), ragged ones (17: a node-cell covered by
# three point blocks' windows across the periodic seam) and a grid of whole point blocks,
# two per axis (16)
@pytest.mark.parametrize("nx,ny,seed,scheme", [(6, 5, 1, "tai"), (7, 8, 2, "tai"), (6, 5, 3, "rb"), (7, 8, 4, "rb"),
                                               (13, 11, 5, "tai"), (17, 12, 6, "tai"), (17, 12, 7, "rb"),
                                               (16, 16, 8, "tai"), (16, 16, 9, "rb"), (24, 17, 10, "tai")])
def test_adjoint_exact_vs_oracle_jacobian(torch_dev, orc, nx, ny, seed, scheme):
    P = I.random_smooth(nx, ny, seed=seed, amp=0.15, vel=(0.35, -0.25))
    s0 = P.state()
    # RB is stable only up to nu ~ 0.195 (Sec. 5.2); the Jacobian does not care, but
    # keep both schemes at a step the paper runs them at
    dt = P.dt_for_cfl(0.45 if scheme == "tai" else 0.19)
    sch = 0 if scheme == "tai" else 1
    n = s0.size
    rng = np.random.default_rng(seed)
    lam = rng.normal(size=s0.shape)
    # (J^T lambda)_k = (J e_k) . lambda, one column of the oracle's Jacobian at a time
    want = np.zeros(n)
    e = np.zeros(n)
    for k in range(n):
        e[:] = 0.0
        e[k] = 1.0
        _, jv = orc.step_jvp(s0, e.reshape(s0.shape), P.h, P.gamma, dt, scheme=sch, threads=1)
        want[k] = jv.ravel() @ lam.ravel()
    want = want.reshape(s0.shape)
    got = gpu_adjoint(torch_dev, P, s0, lam, dt, scheme)
    err = np.abs(got - want).max() / np.abs(want).max()
    print("adjoint vs oracle J^T lambda:", scheme, "max rel", err)
    assert err < 1e-11


@pytest.mark.parametrize("scheme", ["tai", "rb"])
def test_adjoint_dot_product(torch_dev, orc, scheme):
    P = I.isentropic_vortex(32, uinf=(1.0, 1.0))
    s0 = P.state()
    dt = P.dt_for_cfl(0.4 if scheme == "tai" else 0.19)
    rng = np.random.default_rng(7)
    for _ in range(3):
        v = rng.normal(size=s0.shape)
        lam = rng.normal(size=s0.shape)
        _, jv = orc.step_jvp(s0, v, P.h, P.gamma, dt, scheme=0 if scheme == "tai" else 1)
        lhs = float(np.sum(lam * jv))
        rhs = float(np.sum(gpu_adjoint(torch_dev, P, s0, lam, dt, scheme) * v))
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.sqrt(np.sum(lam ** 2) * np.sum(jv ** 2)) * 1e-3)


def test_rollout_gradient_vs_fd(torch_dev):
    """Gradient of a quadratic functional of the final state w.r.t. the initial
    density planes through 40 steps (checkpoints every 8) against central FD."""
    torch, dev = torch_dev
    from paper_2605_12915_amd.autodiff import rollout
    from paper_2605_12915_amd.stepper import Stepper
    P = I.acoustic_pulse_adjoint(48, width=0.15)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    x0 = torch.from_numpy(s0).to(dev)
    w = torch.from_numpy(np.random.default_rng(3).normal(size=s0.shape)).to(dev)

    def J(x):
        return torch.sum(w * (rollout(x, st, dt, 40, 8) - x0) ** 2)

    x = x0.clone().requires_grad_(True)
    val = J(x)
    val.backward()
    grad = x.grad.detach()
    rho_planes = [0, 4, 8, 12]
    rng = np.random.default_rng(11)
    for _ in range(3):
        d = torch.zeros_like(x0)
        for p in rho_planes:
            d[p] = torch.from_numpy(rng.normal(size=s0.shape[1:])).to(dev)
        eps = 1e-6
        with torch.no_grad():
            fd = (J(x0 + eps * d) - J(x0 - eps * d)) / (2 * eps)
        ad = torch.sum(grad * d)
        rel = abs(float(fd - ad)) / max(abs(float(ad)), 1e-30)
        print("rollout FD check: ad", float(ad), "fd", float(fd), "rel", rel)
        assert rel < 1e-6


def test_config4_gradient_vs_fd_512(torch_dev):
    """The differentiation workload at full size: 512^2 Gaussian acoustic pulse with
    seeded centre jitter, 200 steps at CFL 0.4 with checkpoints every 20, gradient of
    the acoustic energy in the annulus 0.10 <= r <= 0.20 (cell-average primitives)
    with respect to the four initial density planes, against central differences in 8
    random directions of that subspace.  Bar: relative error <= 1e-6 per direction at
    the step eps = u^(1/3) max|rho| that balances truncation against rounding (u the
    unit roundoff); at eps = 1e-6 max|rho| the rounding of the 200-step functional
    dominates in directions with small derivatives, so there the bar is 1e-6 of
    |grad| |d| (the normwise form)."""
    torch, dev = torch_dev
    from paper_2605_12915_amd.autodiff import rollout
    from paper_2605_12915_amd.stepper import Stepper
    n, steps, every = 512, 200, 20
    P = I.acoustic_pulse_adjoint(n)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    g = P.gamma
    st = Stepper(P.nx, P.ny, P.h, g, device=dev)
    x0 = torch.from_numpy(s0).to(dev)
    c = (np.arange(n) + 0.5) * P.h
    X, Y = np.meshgrid(c, c)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2)
    mask = torch.from_numpy(((r >= 0.10) & (r <= 0.20)).astype(np.float64)).to(dev)
    rho0, p0 = P.bg[0], P.bg[3]
    c0sq = g * p0 / rho0

    def J(x):
        U = x[:4]
        rho = U[0]
        u, v = U[1] / rho, U[2] / rho
        p = (g - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
        e = (p - p0) ** 2 / (2.0 * rho0 * c0sq) + 0.5 * rho0 * (u * u + v * v)
        return P.h * P.h * torch.sum(mask * e)

    def J_plain(x):
        z = x.clone()
        st.step(z, dt, steps)
        return float(J(z))

    xg = x0.clone().requires_grad_(True)
    J(rollout(xg, st, dt, steps, every)).backward()
    G = xg.grad.detach()
    rho_planes = [0, 4, 8, 12]
    scale = float(x0[rho_planes].abs().max())
    gnorm = float(G[rho_planes].norm())
    rng = np.random.default_rng(8)
    eps_opt, eps6 = np.cbrt(np.finfo(np.float64).eps) * scale, 1e-6 * scale
    with torch.no_grad():
        for k in range(8):
            d = torch.zeros_like(x0)
            for pl in rho_planes:
                d[pl] = torch.from_numpy(rng.normal(size=s0.shape[1:])).to(dev)
            ad = float(torch.sum(G * d))
            fd = (J_plain(x0 + eps_opt * d) - J_plain(x0 - eps_opt * d)) / (2.0 * eps_opt)
            fd6 = (J_plain(x0 + eps6 * d) - J_plain(x0 - eps6 * d)) / (2.0 * eps6)
            rel = abs(fd - ad) / abs(ad)
            nrm6 = abs(fd6 - ad) / (gnorm * float(d.norm()))
            print(f"direction {k}: ad {ad:.12e} rel err {rel:.2e} (eps {eps_opt:.1e}), "
                  f"{abs(fd6 - ad) / abs(ad):.2e} / normwise {nrm6:.2e} (eps {eps6:.1e})", flush=True)
            assert rel <= 1e-6
            assert nrm6 <= 1e-6


@pytest.mark.parametrize("scheme", ["tai", "rb"])
def test_rollout_gradient_vs_oracle_jvp(torch_dev, orc, scheme):
    """The checkpointed rollout's gradient (autograd through 30 steps, checkpoints every
    7, so the last segment is short) against the oracle's own derivative: the
    complex-step JVP chained through the same 30 steps gives <w, J_30 v>, which must
    equal <grad of <w, state_30>, v> for random w and v (all 16 planes)."""
    torch, dev = torch_dev
    from paper_2605_12915_amd.autodiff import rollout
    from paper_2605_12915_amd.stepper import Stepper
    P = I.random_smooth(24, 20, seed=31, amp=0.1, vel=(0.3, 0.2))
    s0 = P.state()
    dt = P.dt_for_cfl(0.45 if scheme == "tai" else 0.19)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme=scheme, device=dev)
    rng = np.random.default_rng(32)
    w = rng.normal(size=s0.shape)
    v = rng.normal(size=s0.shape)
    x = torch.from_numpy(s0).to(dev).requires_grad_(True)
    torch.sum(torch.from_numpy(w).to(dev) * rollout(x, st, dt, 30, 7)).backward()
    lhs = float(np.sum(x.grad.cpu().numpy() * v))
    sc, tc = s0, v
    for _ in range(30):
        sc, tc = orc.step_jvp(sc, tc, P.h, P.gamma, dt, scheme=0 if scheme == "tai" else 1)
    rhs = float(np.sum(w * tc))
    print(scheme, "rollout <grad, v>", lhs, "oracle <w, J v>", rhs)
    assert abs(lhs - rhs) <= 1e-11 * np.sqrt(np.sum(w * w) * np.sum(tc * tc))


@pytest.mark.parametrize("scheme", ["tai", "rb"])
def test_adjoint_pulse_512_dot_product(torch_dev, orc, scheme):
    """512^2 acoustic pulse of the gradient benchmark: <lambda, J v> from the oracle's
    complex-step JVP equals <J^T lambda, v> from the GPU adjoint (RB at a step it is
    stable at)."""
    P = I.acoustic_pulse_adjoint(512)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4 if scheme == "tai" else 0.19)
    rng = np.random.default_rng(12)
    v = rng.normal(size=s0.shape)
    lam = rng.normal(size=s0.shape)
    _, jv = orc.step_jvp(s0, v, P.h, P.gamma, dt, scheme=0 if scheme == "tai" else 1)
    lhs = float(np.sum(lam * jv))
    rhs = float(np.sum(gpu_adjoint(torch_dev, P, s0, lam, dt, scheme) * v))
    print("512^2 pulse dot product", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-10 * np.sqrt(np.sum(lam ** 2) * np.sum(jv ** 2))


@pytest.mark.parametrize("scheme", ["tai", "rb"])
def test_adjoint_repeated_calls_on_one_context(torch_dev, scheme):
    """A context's adjoint scratch (recomputed intermediates, reverse accumulators) carries
    nothing from one call to the next: consecutive calls on one context (different states
    and cotangents, forward steps in between; a ragged 37 x 29 grid and a 48 x 32 one of
    whole point blocks) equal calls on fresh contexts, up to the order of the atomic
    additions."""
    torch, dev = torch_dev
    from paper_2605_12915_amd.stepper import Stepper
    for nx, ny in ((37, 29), (48, 32)):
        _repeated_calls(torch, dev, Stepper, scheme, nx, ny)


def _repeated_calls(torch, dev, Stepper, scheme, nx, ny):
    P = I.random_smooth(nx, ny, seed=21, amp=0.15, vel=(0.3, -0.2))
    dt = P.dt_for_cfl(0.45 if scheme == "tai" else 0.19)
    rng = np.random.default_rng(22)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme=scheme, device=dev)
    x = torch.from_numpy(P.state()).to(dev)
    for call in range(4):
        lam = rng.normal(size=P.state().shape) * (10.0 if call % 2 else 1.0)
        s0 = x.cpu().numpy()
        got = st.adjoint(x, torch.from_numpy(lam).to(dev), dt).cpu().numpy()
        want = gpu_adjoint((torch, dev), P, s0, lam, dt, scheme)
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err < 1e-13, (nx, ny, call, err)
        st.step(x, dt, 2)
