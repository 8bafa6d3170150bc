"""Drivers for the paper's numerical experiments on the GPU step (Sec. 4.2 mixed
wave packet; Sec. 6 isentropic vortex convergence and CFL sweep, acoustic pulse,
low-Mach shear, Kelvin-Helmholtz robustness).

Every driver steps a seeded analytic initial condition (inputs.py) with the HIP
step through the C ABI and reads the FP64 diagnostics (af_diagnostics) along the
way; nothing here computes any part of the step.  The time step follows the
paper's CFL definition, dt = CFL h / max(|u| + c), re-evaluated from the current
state every `every` steps, the last step shortened to land on t_end.
"""
from __future__ import annotations

import math
import time
from typing import Optional

import numpy as np
import torch

from . import inputs as I
from .stepper import Stepper


def run(P: I.Problem, t_end: float, cfl: float, scheme: str = "tai", every: int = 10,
        check_errors: bool = True, device: Optional[torch.device] = None) -> dict:
    """Advance problem P to t_end.  Returns the final state (FP64 tensor on the
    device), the number of steps, the wall time and the diagnostics history
    [(t, diag dict)] sampled every `every` steps (first and last included)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme=scheme, check_errors=check_errors, device=dev)
    x = torch.from_numpy(P.state()).to(dev)
    t, nsteps = 0.0, 0
    d = st.diagnostics(x, 0.0)
    hist = [(0.0, d)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    while t < t_end:
        dt = cfl * P.h / d["max_speed"]
        rest = t_end - t
        last = rest <= every * dt
        if last:                       # n equal steps, no larger than dt, that end on t_end
            n = max(1, int(math.ceil(rest / dt - 1e-9)))
            dt = rest / n
        else:
            n = every
        st.step(x, dt, n)
        t = t_end if last else t + n * dt
        nsteps += n
        d = st.diagnostics(x, dt)
        hist.append((t, d))
    torch.cuda.synchronize(dev)
    return {"problem": P.name, "nx": P.nx, "ny": P.ny, "t": t, "steps": nsteps, "state": x,
            "seconds": time.perf_counter() - t0, "history": hist, "stepper": st}


def mixed_packet(n: int = 56, t_end: float = 1.0, nu: float = 0.25, scheme: str = "tai",
                 device: Optional[torch.device] = None) -> dict:
    """Sec. 4.2: the linearised mixed packet (entropy, shear and two acoustic waves,
    amplitudes 1e-6) against its exact solution, at the acoustic CFL nu = c0 dt / h with
    N = round(t_end / dt) equal steps (56^2, nu = 0.25: 265 steps, t = 0.99995); the
    largest point-value and average errors relative to the amplitude."""
    P, at = I.mixed_packet(n)
    c0 = math.sqrt(P.gamma * P.bg[3] / P.bg[0])
    dt = nu * P.h / c0
    steps = max(1, int(round(t_end / dt)))
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    st = Stepper(P.nx, P.ny, P.h, P.gamma, scheme=scheme, check_errors=True, device=dev)
    x = torch.from_numpy(P.state()).to(dev)
    st.step(x, dt, steps)
    t = steps * dt
    exact = I.make_state(at(t), n, n, 0.0, 0.0, P.h, P.gamma)
    got = x.cpu().numpy()
    return {"n": n, "nu": nu, "dt": dt, "steps": steps, "t": t, "scheme": scheme, "state": x,
            "point_error_over_amplitude": float(np.abs(got[4:] - exact[4:]).max()) / 1e-6,
            "average_error_over_amplitude": float(np.abs(got[:4] - exact[:4]).max()) / 1e-6}


def mixed_packet_refinement(ns=(16, 32, 64, 128), nu: float = 0.25, scheme: str = "tai", **kw) -> dict:
    """Sec. 4.2 refinement at fixed nu to t ~ 1: point-value errors per grid and the
    observed orders (the paper: third order for the transported update, second for
    the additive one)."""
    rows = []
    for n in ns:
        r = mixed_packet(n, 1.0, nu, scheme, **kw)
        rows.append({k: r[k] for k in ("n", "steps", "t", "point_error_over_amplitude", "average_error_over_amplitude")})
    orders = [math.log(a["point_error_over_amplitude"] / b["point_error_over_amplitude"]) / math.log(b["n"] / a["n"])
              for a, b in zip(rows, rows[1:])]
    return {"rows": rows, "orders": orders}


def pulse_asymmetry(n: int = 80, t_end: float = 2.5, cfl: float = 0.475, **kw) -> dict:
    """Sec. 6, acoustic pulse on [-4, 4]^2: the exact solution is radially symmetric;
    reports the vertex pressures' largest deviation under the transposition and the
    two mirror symmetries of the grid, relative to the pulse amplitude."""
    P = I.paper_pulse(n)
    r = run(P, t_end, cfl, **kw)
    p = r["state"][7].cpu().numpy()                     # vertex pressure, [j][i], vertex i at x = -4 + i h
    flip = lambda a, ax: np.roll(np.flip(a, ax), 1, ax)  # x -> -x on vertices (index i -> -i mod n)
    r["asymmetry"] = float(max(np.abs(p - p.T).max(), np.abs(p - flip(p, 0)).max(), np.abs(p - flip(p, 1)).max()))
    r["amplitude"] = float(p.max() - p.min())
    return r


def radial_asymmetry(state: np.ndarray, n: int) -> float:
    """Largest spread of the pressure among point nodes at the same distance from the
    centre of the [-L/2, L/2]^2 grid (n even; vertex, vertical- and horizontal-edge nodes
    together, distances compared exactly in half-cell units).  Nodes that are images of
    each other under the grid's symmetries agree to round-off, so the spread measures
    the direction dependence of the solution: zero for an exactly radial field."""
    c = n // 2
    idx = 2 * (np.arange(n, dtype=np.int64) - c)
    R2, p = [], []
    for plane, ox, oy in ((7, 0, 0), (11, 0, 1), (15, 1, 0)):
        X = idx[None, :] + ox
        Y = idx[:, None] + oy
        R2.append((X * X + Y * Y).ravel())
        p.append(np.asarray(state[plane]).ravel())
    R2, p = np.concatenate(R2), np.concatenate(p)
    order = np.argsort(R2, kind="stable")
    R2, p = R2[order], p[order]
    starts = np.flatnonzero(np.r_[True, R2[1:] != R2[:-1]])
    return float((np.maximum.reduceat(p, starts) - np.minimum.reduceat(p, starts)).max())


def pulse_refinement(ns=(80, 160, 320), ref_n: int = 640, t_end: float = 2.5, cfl: float = 0.475,
                     scheme: str = "tai", **kw) -> dict:
    """Sec. 6 acoustic pulse under refinement (dx = 8 / n): the largest radial asymmetry
    of the point pressures and the largest vertex-pressure error against the ref_n^2
    solution of the same scheme (the paper's reference), both relative to the initial
    pressure amplitude, with observed orders between consecutive grids."""
    def final(n):
        P = I.paper_pulse(n)
        r = run(P, t_end, cfl, scheme=scheme, every=50, **kw)
        return P, r["state"].cpu().numpy()

    Pr, ref = final(ref_n)
    s0 = Pr.state()
    amp = float(s0[7].max() - s0[7].min())
    rows = []
    for n in ns:
        P, st = final(n)
        k = ref_n // n
        err = float(np.abs(st[7] - ref[7][::k, ::k]).max()) / amp
        rows.append({"n": n, "dx": P.h, "asymmetry": radial_asymmetry(st, n) / amp, "max_error": err})
    orders = [{"asymmetry": math.log2(a["asymmetry"] / b["asymmetry"]), "max_error": math.log2(a["max_error"] / b["max_error"])}
              for a, b in zip(rows, rows[1:])]
    return {"rows": rows, "orders": orders, "reference_n": ref_n,
            "reference_asymmetry": radial_asymmetry(ref, ref_n) / amp}


def low_mach_shear(nx: int = 64, t_end: float = 80.0, cfl: float = 0.45, **kw) -> dict:
    """Sec. 6, low Mach number shear (M = 1e-2) on [0, 2] x [-0.5, 0.5]: time histories
    of the vorticity integral (zero up to round-off), the enstrophy, the entropy
    functional and the conserved totals."""
    P = I.low_mach_shear(nx)
    r = run(P, t_end, cfl, **kw)
    H = r["history"]
    r["max_abs_vorticity_integral"] = max(abs(d["vorticity"]) for _, d in H)
    e0 = H[0][1]["enstrophy"]
    r["enstrophy_ratio_final"] = H[-1][1]["enstrophy"] / e0
    m0 = H[0][1]["mass"]
    r["max_mass_drift"] = max(abs(d["mass"] - m0) for _, d in H) / abs(m0)
    return r


def kelvin_helmholtz(n: int = 64, t_end: float = 15.0, cfl: float = 0.475, **kw) -> dict:
    """Sec. 6 robustness test on [-1, 1]^2 to t = 15 without limiters: completes when
    no step raised a non-physical, foot or acoustic-CFL status (AF_CHECK)."""
    P = I.kelvin_helmholtz(n)
    r = run(P, t_end, cfl, **kw)
    H = r["history"]
    r["min_rho"] = min(d["min_rho"] for _, d in H)
    r["min_p"] = min(d["min_p"] for _, d in H)
    return r


def paper_vortex(n: int) -> I.Problem:
    """Sec. 6, isentropic vortex: [0, 10] x [-5, 5], centre (5, 0), beta = 5, carried by
    (u, v) = (1, 0); after t = 10 (one period) the exact solution is the initial data."""
    return I.isentropic_vortex(n, center=(5.0, 0.0), uinf=(1.0, 0.0), y0=-5.0)


def vortex_error(n: int, cfl: float, scheme: str = "tai", t_end: float = 10.0, **kw) -> dict:
    """One period of the vortex at the given CFL: L2 (sqrt(h^2 sum e^2)) and L-inf errors
    of the density averages against the exact ones.  An unstable run (a non-physical
    state or a foot or acoustic-CFL violation raised by the step's checks) is reported
    with stable = False instead of errors."""
    from ._lib import AfError
    P = paper_vortex(n)
    exact = P.state()[0]
    try:
        r = run(P, t_end, cfl, scheme=scheme, every=50, **kw)
    except AfError as e:
        return {"n": n, "cfl": cfl, "scheme": scheme, "stable": False, "error": str(e)}
    e = r["state"][0].cpu().numpy() - exact
    if not np.isfinite(e).all():
        return {"n": n, "cfl": cfl, "scheme": scheme, "stable": False, "error": "non-finite state"}
    return {"n": n, "cfl": cfl, "scheme": scheme, "stable": True, "steps": r["steps"],
            "l2": float(math.sqrt(P.h * P.h * float(np.sum(e * e)))), "linf": float(np.abs(e).max())}


def vortex_convergence(ns=(16, 32, 64, 128), cfl: float = 0.3, scheme: str = "tai", **kw) -> dict:
    """Sec. 6 grid-refinement study of the vortex at CFL 0.3: errors per grid and the
    observed orders between consecutive grids."""
    rows = [vortex_error(n, cfl, scheme, **kw) for n in ns]
    orders = []
    for a, b in zip(rows, rows[1:]):
        orders.append({"l2": math.log(a["l2"] / b["l2"]) / math.log(b["n"] / a["n"]),
                       "linf": math.log(a["linf"] / b["linf"]) / math.log(b["n"] / a["n"])})
    return {"rows": rows, "orders": orders}


def vortex_cfl_sweep(n: int = 64, cfls=(0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0),
                     scheme: str = "tai", **kw) -> list:
    """Sec. 6 CFL sweep of the vortex on one grid: error (or instability) per CFL."""
    return [vortex_error(n, c, scheme, **kw) for c in cfls]


def _main(argv=None) -> int:
    """python -m paper_2605_12915_amd.experiments NAME [--scheme tai|rb]: run one
    experiment with its default settings and print its results as one JSON line."""
    import argparse
    import json
    ap = argparse.ArgumentParser(prog="python -m paper_2605_12915_amd.experiments")
    ap.add_argument("name", choices=["mixed_packet", "mixed_packet_refinement", "vortex_convergence",
                                     "vortex_cfl_sweep", "pulse_asymmetry", "pulse_refinement",
                                     "low_mach_shear", "kelvin_helmholtz"])
    ap.add_argument("--scheme", default="tai", choices=["tai", "rb"])
    a = ap.parse_args(argv)
    fn = globals()[a.name]
    kw = {"scheme": a.scheme}
    # RB is linearly unstable above an acoustic CFL of ~0.195 (Sec. 5.2): the paper's
    # RB settings where the default CFL is higher
    rb_cfl = {"kelvin_helmholtz": 0.25, "pulse_asymmetry": 0.2, "pulse_refinement": 0.2, "low_mach_shear": 0.19}
    if a.scheme == "rb" and a.name in rb_cfl:
        kw["cfl"] = rb_cfl[a.name]
    r = fn(**kw)

    def plain(v):
        if isinstance(v, dict):
            return {k: plain(x) for k, x in v.items() if k not in ("state", "stepper", "history")}
        if isinstance(v, (list, tuple)):
            return [plain(x) for x in v]
        if isinstance(v, (np.floating, np.integer)):
            return v.item()
        return v

    out = plain(r)
    if isinstance(r, dict) and "history" in r:
        out["history"] = [{"t": t, **d} for t, d in r["history"]]
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
