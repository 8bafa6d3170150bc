"""Benchmark of the RB-TAI Active Flux step on one MI355X.

Headline (N = 1): periodic 2048 x 2048 grid, FP64, background rho = 1, p = 1/1.4,
(u, v) = (0.5, 0.3) plus 16 seeded Fourier modes per primitive field (wavenumbers
up to 8, amplitude 1e-3), CFL 0.4.  Inputs are generated on the host and copied to
HBM before the timed region; K steps are timed between two device synchronisations.

The same run measures the three forms built on the step (in "forms"):
  fp32     4096^2 isentropic vortex and 4096^2 Gaussian pulse, 500 FP32 steps each,
           throughput and per-field error against the FP64 GPU path;
  adjoint  512^2 acoustic pulse: adjoint-step / forward-step time, the full gradient
           of an annulus acoustic energy through 200 steps (checkpoints every 20)
           and its central finite-difference check in 8 density directions;
  batch    64 double shear layers of seeded sizes N in [32, 1024], 1000 FP32 steps
           in one hipGraph (one launch per step; tile shape and grid mode autotuned);
           aggregate rate, tuning table, per-size-class rates, error against FP64;
  fc       the foot-centred exact point update (App. C) on the 256^2 Fourier-mode
           flow: step rate, its cost against the transported step at the same size.

Prints ONE JSON line; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PLANE_NAMES = [f"{fam}.{v}" for fam, vs in (("avg", ("rho", "rhou", "rhov", "E")), ("V", ("rho", "u", "v", "p")),
                                              ("EV", ("rho", "u", "v", "p")), ("EH", ("rho", "u", "v", "p")))
               for v in vs]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--fc-n", type=int, default=256)
    ap.add_argument("--fc-steps", type=int, default=3)
    ap.add_argument("--forms", default="fp32,adjoint,batch,fc",
                    help="comma list of forms to measure after the headline (or 'none')")
    ap.add_argument("--fp32-n", type=int, default=4096)
    ap.add_argument("--fp32-steps", type=int, default=500)
    ap.add_argument("--adj-n", type=int, default=512)
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-lite", action="store_true",
                    help="batch form without the one-by-one comparison and the size classes")
    ap.add_argument("--adj-dirs", type=int, default=8, help="finite-difference directions of the gradient check")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed repeats of the K headline steps; the median repeat is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=0,
                    help="grid of the oracle sample (0: the headline grid and state itself)")
    ap.add_argument("--cpu-sample-steps", type=int, default=8)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(n: int, steps: int, P=None, s=None):
    """The oracle as it stands, on the host cores, over a bounded sample of the
    workload: the headline grid and state (P, s) for a few steps, or an n x n grid of
    the same flow."""
    from oracle import ref
    from paper_2605_12915_amd import inputs as I
    if P is None:
        P = I.fourier_modes(n)
        s = P.state()
    n = P.nx
    dt = P.dt_for_cfl(0.4)
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref.run(s, P.h, P.gamma, dt, steps, threads=threads)
    el = time.perf_counter() - t0
    # one thread, on a 256^2 grid of the same flow (a second or two)
    Q = I.fourier_modes(256)
    q = Q.state()
    t1 = time.perf_counter()
    ref.run(q, Q.h, Q.gamma, Q.dt_for_cfl(0.4), 2, threads=1)
    el1 = time.perf_counter() - t1
    return {"value": n * n * steps / el / 1e6, "unit": "Mcell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} Fourier-mode flow, {steps} steps, FP64, {threads} OpenMP threads, {el:.2f} s",
            "single_thread_value": 256 * 256 * 2 / el1 / 1e6,
            "single_thread_sample": f"256x256, 2 steps, 1 thread, {el1:.2f} s"}


def timed(torch, fn):
    """Wall time of fn() between two device synchronisations."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


# ---------------------------------------------------------------------------------
# FP32 precision form
# ---------------------------------------------------------------------------------
def abs_from_pert(torch, x32, bg, gamma):
    """FP32 perturbation planes -> absolute FP64 planes (on the device)."""
    from paper_2605_12915_amd.stepper import background_cons
    off = list(background_cons(bg, gamma)) + [float(b) for b in bg] * 3
    return x32.double() + torch.tensor(off, dtype=torch.float64, device=x32.device)[:, None, None]


def fp32_roofline(perf, kname, ach, ker_ms, ncell):
    """FP32 roofline of one launch: algorithmic flops / kernel time against the FP32
    vector peak, with the stored counter figures of that kernel when they are current
    (HBM bytes, executed FP32 flops)."""
    roof = {"bound": "alu", "achieved": ach, "peak": perf.FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / perf.FP32_PEAK_TFLOPS, "kernel": kname, "kernel_ms": ker_ms,
            "algo_flops_per_cell": perf.ALGO_FLOPS_PER_CELL_F64, "algo_bytes_per_cell": perf.ALGO_BYTES_PER_CELL_F32,
            "hbm_gbs_algorithmic": perf.ALGO_BYTES_PER_CELL_F32 * ncell / (ker_ms * 1e-3) / 1e9, "traffic": None}
    tr = perf.stored_traffic(kname)
    if tr and tr.get("cells_per_launch") == ncell:
        roof["traffic"] = tr["traffic_bytes_per_launch"]
        roof["traffic_gbs"] = tr["traffic_bytes_per_launch"] / (ker_ms * 1e-3) / 1e9
        roof["traffic_frac_of_peak"] = roof["traffic_gbs"] / perf.HBM_PEAK_GBS
        if tr.get("executed_fp32_flops_per_launch"):
            ex = tr["executed_fp32_flops_per_launch"] / (ker_ms * 1e-3) / 1e12
            roof.update({"executed_tflops": ex, "executed_frac_of_peak": ex / perf.FP32_PEAK_TFLOPS})
    return roof


def form_fp32(torch, dev, n, steps):
    from paper_2605_12915_amd import inputs as I
    from paper_2605_12915_amd import perf
    from paper_2605_12915_amd.stepper import Stepper, to_perturbation
    out = {}
    for tag, P in (("isentropic_vortex", I.isentropic_vortex(n, uinf=(1.0, 1.0))),
                   ("gaussian_pulse", I.gaussian_pulse(n, amp=0.1, width=0.05))):
        log(f"fp32 {tag}: generating {n}x{n} input")
        s0 = P.state()
        dt = P.dt_for_cfl(0.4)
        ncell = P.nx * P.ny
        # FP64 reference on the GPU (its parity with the oracle is the FP64 tests' bar)
        st64 = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
        x64 = torch.from_numpy(s0).to(dev)
        el64 = timed(torch, lambda: st64.step(x64, dt, steps))
        st64.close()
        st32 = Stepper(P.nx, P.ny, P.h, P.gamma, precision="f32", bg=P.bg, device=dev)
        x32 = torch.from_numpy(to_perturbation(s0, P.bg, P.gamma)).to(dev)
        del s0
        st32.step(x32.clone(), dt, 3)                       # warm-up on a copy
        el32 = timed(torch, lambda: st32.step(x32, dt, steps))
        status = st32.read_status()
        _, ker_ms = st32.time_steps(x32, dt, 20)
        kname = st32.dominant_kernel()
        st32.close()
        got = abs_from_pert(torch, x32, P.bg, P.gamma)
        del x32
        per = {}
        worst_l2 = worst_linf = 0.0
        for k in range(16):
            r = x64[k]
            e = got[k] - r
            l2 = float(torch.linalg.vector_norm(e) / max(float(torch.linalg.vector_norm(r - r.mean())), 1e-300))
            linf = float(e.abs().max() / max(float(r.max() - r.min()), 1e-300))
            per[PLANE_NAMES[k]] = {"l2_rel": l2, "linf_rel": linf}
            worst_l2, worst_linf = max(worst_l2, l2), max(worst_linf, linf)
        del got, x64
        torch.cuda.empty_cache()
        flops = perf.ALGO_FLOPS_PER_CELL_F64 * ncell
        ach = flops / (ker_ms * 1e-3) / 1e12
        out[tag] = {
            "nx": P.nx, "ny": P.ny, "steps": steps, "dt": dt, "status": status,
            "value": ncell * steps / el32 / 1e6, "unit": "Mcell-updates/s",
            "fp64_value": ncell * steps / el64 / 1e6, "speedup_vs_fp64": el64 / el32,
            "kernel": kname, "kernel_ms": ker_ms,
            "roofline": fp32_roofline(perf, kname, ach, ker_ms, ncell),
            "error_vs_fp64": {"max_l2_rel": worst_l2, "max_linf_rel": worst_linf,
                              "definition": "per plane: ||e||_2 / ||ref - mean(ref)||_2 and max|e| / range(ref)",
                              "per_plane": per},
        }
        log(f"fp32 {tag}: {out[tag]['value']:.0f} Mcell/s, max linf_rel {worst_linf:.2e}")
    return out


# ---------------------------------------------------------------------------------
# Differentiation form
# ---------------------------------------------------------------------------------
def form_adjoint(torch, dev, n, steps, every=20, ndir=8):
    import numpy as np

    from paper_2605_12915_amd import inputs as I
    from paper_2605_12915_amd import perf
    from paper_2605_12915_amd.autodiff import rollout
    from paper_2605_12915_amd.stepper import Stepper
    P = I.acoustic_pulse_adjoint(n)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    g = P.gamma
    st = Stepper(P.nx, P.ny, P.h, g, device=dev)
    x0 = torch.from_numpy(s0).to(dev)
    # per-call times of the forward step and the adjoint step (same state)
    K = 50
    y = torch.empty_like(x0)
    cot = torch.from_numpy(np.random.default_rng(1).normal(size=s0.shape)).to(dev)
    gout = torch.empty_like(x0)
    st.step_out(x0, dt, y)
    st.adjoint(x0, cot, dt, gout)
    t_fwd = timed(torch, lambda: [st.step_out(x0, dt, y) for _ in range(K)]) / K
    t_adj = timed(torch, lambda: [st.adjoint(x0, cot, dt, gout) for _ in range(K)]) / K

    # the same two sequences between HIP events on the stream the library launches on
    # (the context borrows torch's current stream)
    def ev_ms(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / K

    ev_fwd = ev_ms(lambda: [st.step_out(x0, dt, y) for _ in range(K)])
    ev_adj = ev_ms(lambda: [st.adjoint(x0, cot, dt, gout) for _ in range(K)])
    ncell = P.nx * P.ny
    ach = perf.ALGO_FLOPS_PER_CELL_ADJ * ncell / (ev_adj * 1e-3) / 1e12
    t_alu = perf.ALGO_FLOPS_PER_CELL_ADJ * ncell / (perf.FP64_PEAK_TFLOPS * 1e12)
    t_hbm = perf.ALGO_BYTES_PER_CELL_ADJ * ncell / (perf.HBM_PEAK_GBS * 1e9)
    roof = {"bound": "alu" if t_alu >= t_hbm else "hbm", "achieved": ach, "peak": perf.FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / perf.FP64_PEAK_TFLOPS, "kernels": perf.ADJOINT_KERNELS,
            "step_ms_events": ev_adj, "algo_flops_per_cell": perf.ALGO_FLOPS_PER_CELL_ADJ,
            "algo_bytes_per_cell": perf.ALGO_BYTES_PER_CELL_ADJ,
            "hbm_gbs_algorithmic": perf.ALGO_BYTES_PER_CELL_ADJ * ncell / (ev_adj * 1e-3) / 1e9,
            "t_alu_ms": t_alu * 1e3, "t_hbm_ms": t_hbm * 1e3, "traffic": None}
    tr = perf.stored_traffic_sum(perf.ADJOINT_KERNELS)
    if tr:
        roof["traffic"] = tr["traffic_bytes_per_launch"]
        roof["traffic_gbs"] = tr["traffic_bytes_per_launch"] / (ev_adj * 1e-3) / 1e9
        if tr.get("executed_fp64_flops_per_launch"):
            ex = tr["executed_fp64_flops_per_launch"] / (ev_adj * 1e-3) / 1e12
            roof.update({"executed_tflops": ex, "executed_frac_of_peak": ex / perf.FP64_PEAK_TFLOPS})
    # annulus acoustic energy from cell-average primitives
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

    def J_of_initial(x):
        z = x.clone()
        st.step(z, dt, steps)
        return float(J(z))

    xg = x0.clone().requires_grad_(True)

    def grad():
        val = J(rollout(xg, st, dt, steps, every))
        val.backward()
        return val

    grad()                                   # first use loads torch's own kernels
    xg.grad = None
    t_grad = timed(torch, grad)

    # the same gradient with every state kept (steps x 16 planes: a few GB at 512^2 against
    # 288 GB of HBM), so that the backward pass recomputes nothing
    def grad_all():
        xa = x0.clone().requires_grad_(True)
        val = J(rollout(xa, st, dt, steps, 1))
        val.backward()
        return xa.grad

    ga = grad_all()
    t_grad_all = timed(torch, grad_all)
    J_of_initial(x0)
    t_fwd_roll = timed(torch, lambda: J_of_initial(x0))
    G = xg.grad.detach()
    rng = np.random.default_rng(8)
    rho_planes = [0, 4, 8, 12]
    scale = float(x0[rho_planes].abs().max())
    # central differences: the step balancing O(eps^2) truncation against O(u / eps)
    # rounding is the cube root of the unit roundoff u (times the variable's scale);
    # 1e-6 of the scale is also reported
    eps_list = [np.cbrt(np.finfo(np.float64).eps) * scale, 1e-6 * scale]
    errs = {e: [] for e in eps_list}
    norm_errs = []
    gnorm = float(G[rho_planes].norm())
    with torch.no_grad():
        for _ in range(ndir):
            d = torch.zeros_like(x0)
            for pl in rho_planes:
                d[pl] = torch.from_numpy(rng.normal(size=s0.shape[1:])).to(dev)
            ad = float(torch.sum(G * d))
            for eps in eps_list:
                fd = (J_of_initial(x0 + eps * d) - J_of_initial(x0 - eps * d)) / (2.0 * eps)
                errs[eps].append(abs(fd - ad) / max(abs(ad), 1e-300))
                if eps == eps_list[0]:
                    norm_errs.append(abs(fd - ad) / (gnorm * float(d.norm())))
    eps = eps_list[0]
    st.close()
    out = {"nx": n, "ny": n, "dt": dt, "forward_step_ms": t_fwd * 1e3, "adjoint_step_ms": t_adj * 1e3,
           "adjoint_over_forward": t_adj / t_fwd, "forward_step_ms_events": ev_fwd, "adjoint_step_ms_events": ev_adj,
           "adjoint_over_forward_events": ev_adj / ev_fwd, "cotangent": "dense, standard normal in every plane",
           "roofline": roof, "gradient_steps": steps, "checkpoint_every": every,
           "gradient_ms": t_grad * 1e3, "forward_rollout_ms": t_fwd_roll * 1e3,
           "gradient_over_forward_rollout": t_grad / t_fwd_roll,
           "gradient_every_state_kept_ms": t_grad_all * 1e3,
           "gradient_every_state_kept_over_forward_rollout": t_grad_all / t_fwd_roll,
           "gradient_every_state_kept_max_rel_diff": float((ga - G).abs().max() / G.abs().max()),
           "fd_check": {"directions": ndir, "eps": eps, "max_rel_err": max(errs[eps]),
                        "max_err_over_grad_norm": max(norm_errs),
                        "eps_1e-6": {"eps": eps_list[1], "max_rel_err": max(errs[eps_list[1]])},
                        "subspace": "the four density planes of the initial state"}}
    log(f"adjoint: ratio {out['adjoint_over_forward']:.2f}, FD max rel {max(errs[eps]):.2e} "
        f"(eps {eps:.2e}; {max(errs[eps_list[1]]):.2e} at eps {eps_list[1]:.2e})")
    return out


# ---------------------------------------------------------------------------------
# Batching form
# ---------------------------------------------------------------------------------
def form_batch(torch, dev, count, steps, big_fp32_rate, lite=False):
    from paper_2605_12915_amd import inputs as I
    from paper_2605_12915_amd import perf
    from paper_2605_12915_amd.stepper import Batch, Stepper, to_perturbation
    sizes = I.batch_sizes(count)
    log(f"batch: generating {count} inputs, {sum(n * n for n in sizes)} cells")
    Ps = [I.double_shear_layer(N) for N in sizes]
    dts = [P.dt_for_cfl(0.4) for P in Ps]
    xs0 = [torch.from_numpy(to_perturbation(P.state(), P.bg, P.gamma)).to(dev) for P in Ps]
    grids = [dict(nx=P.nx, ny=P.ny, h=P.h, gamma=P.gamma, bg=P.bg) for P in Ps]

    def run_batch(idx, nsteps, keep=False):
        b = Batch([grids[k] for k in idx], device=dev)
        xs = [xs0[k].clone() for k in idx]
        b.step(xs, [dts[k] for k in idx], nsteps)          # tuning + capture + first replay
        kept = [x.clone() for x in xs] if keep else None   # exactly nsteps steps from the input
        el = timed(torch, lambda: b.step(xs, [dts[k] for k in idx], nsteps))
        info, status, kname = b.info(), b.read_status(), b.dominant_kernel()
        b.close()
        return sum(sizes[k] ** 2 for k in idx) * nsteps / el / 1e6, el, info, status, kname, kept

    allidx = list(range(count))
    rate, el, info, status, kname, kept = run_batch(allidx, steps, keep=not lite)
    ncells = sum(n * n for n in sizes)
    # one launch per step over every grid: the launch duration is the per-step time of
    # the replayed graph
    launch_ms = el * 1e3 / steps
    ach = perf.ALGO_FLOPS_PER_CELL_F64 * ncells / (launch_ms * 1e-3) / 1e12
    roof = fp32_roofline(perf, kname, ach, launch_ms, ncells)
    if lite:
        return {"instances": count, "cells": ncells, "steps": steps, "value": rate,
                "unit": "Mcell-updates/s", "seconds": el, "status": status, "tuning": info, "roofline": roof}
    # the batch after exactly `steps` steps against the FP64 GPU path on every grid
    # (per plane: L2 and L-inf of the difference over the plane's variation, as in the
    # FP32 form; the worst grid and plane are reported)
    err = {"max_l2_rel": 0.0, "max_linf_rel": 0.0, "worst_grid": None, "worst_plane": None,
           "definition": "per grid and plane: ||e||_2 / ||ref - mean(ref)||_2 and max|e| / range(ref), "
                         "ref = FP64 GPU step from the same initial data"}
    for k, P in enumerate(Ps):
        st64 = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
        x64 = torch.from_numpy(P.state()).to(dev)
        st64.step(x64, dts[k], steps)
        st64.close()
        got = abs_from_pert(torch, kept[k], P.bg, P.gamma)
        for q in range(16):
            r = x64[q]
            e = got[q] - r
            l2 = float(torch.linalg.vector_norm(e) / max(float(torch.linalg.vector_norm(r - r.mean())), 1e-300))
            linf = float(e.abs().max() / max(float(r.max() - r.min()), 1e-300))
            if linf > err["max_linf_rel"]:
                err.update(max_linf_rel=linf, worst_grid=sizes[k], worst_plane=PLANE_NAMES[q])
            err["max_l2_rel"] = max(err["max_l2_rel"], l2)
        del x64, got
    del kept
    # the same instances stepped one by one (one launch per instance and step)
    sts = [Stepper(P.nx, P.ny, P.h, P.gamma, precision="f32", bg=P.bg, device=dev) for P in Ps]
    ys = [x.clone() for x in xs0]
    k1 = max(1, steps // 10)
    for s_, y, dt in zip(sts, ys, dts):
        s_.step(y, dt, 1)
    el1 = timed(torch, lambda: [s_.step(y, dt, k1) for s_, y, dt in zip(sts, ys, dts)])
    for s_ in sts:
        s_.close()
    classes = []
    edges = [32, 64, 128, 256, 512, 1025]
    for lo, hi in zip(edges[:-1], edges[1:]):
        idx = [k for k in allidx if lo <= sizes[k] < hi]
        if not idx:
            continue
        r_, _, inf_, _, _, _ = run_batch(idx, max(100, steps // 5))
        classes.append({"sizes": [lo, hi - 1], "instances": len(idx), "cells": sum(sizes[k] ** 2 for k in idx),
                        "batched_mcells": r_, "tile": inf_["chosen"],
                        "efficiency_vs_large_grid_fp32": r_ / big_fp32_rate if big_fp32_rate else None})
    out = {"instances": count, "sizes_min_max": [min(sizes), max(sizes)], "cells": ncells, "steps": steps,
           "value": rate, "unit": "Mcell-updates/s", "seconds": el, "status": status,
           "launches_per_step": 1, "graph_launches": steps + (steps & 1),
           "tuning": info, "one_by_one_mcells": ncells * k1 / el1 / 1e6,
           "speedup_vs_one_by_one": rate / (ncells * k1 / el1 / 1e6),
           "efficiency_vs_large_grid_fp32": rate / big_fp32_rate if big_fp32_rate else None,
           "size_classes": classes, "roofline": roof, "error_vs_fp64": err}
    log(f"batch: {rate:.0f} Mcell/s aggregate, one-by-one {out['one_by_one_mcells']:.0f}")
    return out


def form_fc(torch, dev, n, steps):
    """The foot-centred exact point update (AF_SCHEME_FC, App. C) against the
    transported update on the same n^2 Fourier-mode flow (the headline's workload at a
    smaller size): HIP-event kernel times of the point kernel and of the transported
    step, their ratio (the paper estimates about a thousand), and the executed-FP64
    roofline of the point kernel from its stored counters (its flops depend on how
    many grid lines cut each disk)."""
    from paper_2605_12915_amd import inputs as I
    from paper_2605_12915_amd import perf
    from paper_2605_12915_amd.stepper import Stepper
    P = I.fourier_modes(n)
    dt = P.dt_for_cfl(0.4)
    x = torch.from_numpy(P.state()).to(dev)
    out = {"nx": n, "ny": n, "steps": steps, "dt": dt, "workload": f"periodic {n}x{n} FP64 Fourier-mode flow, CFL 0.4"}
    for scheme, k in (("fc", steps), ("tai", 50)):
        st = Stepper(n, n, P.h, P.gamma, scheme=scheme, device=dev, check_errors=True)
        st.time_steps(x, dt, 1)
        tot, ker = st.time_steps(x, dt, k)
        out[f"{scheme}_step_ms"] = tot / k
        out[f"{scheme}_kernel_ms"] = ker
        if scheme == "fc":
            kname = st.dominant_kernel()
            y = x.clone()
            st.step(y, dt, 1)
            out["status"] = st.read_status()
            out["finite"] = bool(torch.isfinite(y).all())
        st.close()
    out["value"] = n * n / (out["fc_step_ms"] * 1e-3) / 1e6
    out["unit"] = "Mcell-updates/s"
    out["fc_over_tai_kernel"] = out["fc_kernel_ms"] / out["tai_kernel_ms"]
    out["fc_over_tai_step"] = out["fc_step_ms"] / out["tai_step_ms"]
    roof = {"bound": "alu", "peak": perf.FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "kernel": kname,
            "kernel_ms": out["fc_kernel_ms"], "achieved": None, "frac": None, "traffic": None,
            "achieved_kind": "executed FP64 flops of the point kernel (SQ_INSTS_VALU_FLOPS_FP64 x 64) per launch"}
    tr = perf.stored_traffic(kname)
    if tr and tr.get("cells_per_launch") == n * n and tr.get("executed_fp64_flops_per_launch"):
        ach = tr["executed_fp64_flops_per_launch"] / (out["fc_kernel_ms"] * 1e-3) / 1e12
        roof.update({"achieved": ach, "frac": ach / perf.FP64_PEAK_TFLOPS, "traffic": tr["traffic_bytes_per_launch"],
                     "executed_flops_per_cell": tr["executed_fp64_flops_per_launch"] / (n * n)})
    out["roofline"] = roof
    log(f"fc: {out['value']:.1f} Mcell/s, {out['fc_over_tai_kernel']:.0f}x the transported kernel")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: the step has no multi-GPU path; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_12915_amd import inputs as I
    from paper_2605_12915_amd import perf
    from paper_2605_12915_amd.stepper import Stepper

    dev = torch.device("cuda:0")
    log(f"headline: generating {args.n}x{args.n} input")
    P = I.fourier_modes(args.n)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    x = torch.from_numpy(s0).to(dev)
    torch.cuda.synchronize()
    if args.warmup:
        st.step(x, dt, args.warmup)
    # K steps timed between device synchronisations, repeated; the median repeat is reported
    els = [timed(torch, lambda: st.step(x, dt, args.steps)) for _ in range(max(1, args.repeats))]
    el = sorted(els)[len(els) // 2]
    ncell = P.nx * P.ny
    value = ncell * args.steps / el / 1e6
    # dominant-kernel duration from HIP events on the library's stream
    tot_ms, ker_ms = st.time_steps(x, dt, 20)
    diag = st.diagnostics(x, dt)
    ok = bool(np.isfinite(diag["mass"]))
    t0 = time.perf_counter()
    for _ in range(10):
        st.diagnostics(x, dt)                              # synchronous FP64 reductions
    diag_ms = (time.perf_counter() - t0) * 1e3 / 10
    kname = st.dominant_kernel()
    flops = perf.ALGO_FLOPS_PER_CELL_F64 * ncell            # per launch of the step kernel
    achieved = flops / (ker_ms * 1e-3) / 1e12
    t_alu = flops / (perf.FP64_PEAK_TFLOPS * 1e12)
    t_hbm = perf.ALGO_BYTES_PER_CELL_F64 * ncell / (perf.HBM_PEAK_GBS * 1e9)
    tr = perf.stored_traffic(kname)
    # measured copy bandwidth: a plain 1 GiB device-to-device copy (read + write 2 GiB)
    src = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_s = min(timed(torch, lambda: dst.copy_(src)) for _ in range(5))
    copy_gbs = 2 * src.numel() * 8 / copy_s / 1e9
    del src, dst
    log(f"headline: {value:.0f} Mcell/s, kernel {ker_ms:.3f} ms")
    line = {
        "metric": "Mcell-updates/s per AF step (FP64 vs FP32) at stated error; adjoint/forward ratio",
        "value": value, "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "repeats": len(els),
        "ms_per_step_repeats": [e * 1e3 / args.steps for e in els], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"periodic {P.nx}x{P.ny} FP64 Fourier-mode flow, CFL 0.4, RB-TAI step",
                   "nx": P.nx, "ny": P.ny, "dt": dt},
        "roofline": {"bound": "alu" if t_alu >= t_hbm else "hbm", "achieved": achieved,
                     "peak": perf.FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / perf.FP64_PEAK_TFLOPS,
                     "traffic": tr["traffic_bytes_per_launch"] if tr else None,
                     "kernel": kname, "kernel_ms": ker_ms,
                     "algo_flops_per_cell": perf.ALGO_FLOPS_PER_CELL_F64,
                     "algo_bytes_per_cell": perf.ALGO_BYTES_PER_CELL_F64,
                     "hbm_gbs_algorithmic": perf.ALGO_BYTES_PER_CELL_F64 * ncell / (ker_ms * 1e-3) / 1e9,
                     "t_alu_ms": t_alu * 1e3, "t_hbm_ms": t_hbm * 1e3,
                     "copy_gbs_measured": copy_gbs},
        "finite": ok,
        "diagnostics_ms": diag_ms,
        "value_with_diagnostics_every_step": ncell * args.steps / (el + args.steps * diag_ms * 1e-3) / 1e6,
    }
    if tr:
        # the counters' view of the same kernel: HBM bytes and executed FP64 flops per launch
        gbs = tr["traffic_bytes_per_launch"] / (ker_ms * 1e-3) / 1e9
        line["roofline"].update({"traffic_gbs": gbs, "traffic_frac_of_peak": gbs / perf.HBM_PEAK_GBS,
                                 "traffic_frac_of_copy": gbs / copy_gbs})
        if tr.get("executed_fp64_flops_per_launch"):
            ex = tr["executed_fp64_flops_per_launch"] / (ker_ms * 1e-3) / 1e12
            line["roofline"].update({"executed_tflops": ex, "executed_frac_of_peak": ex / perf.FP64_PEAK_TFLOPS})
    st.close()
    del x
    torch.cuda.empty_cache()
    if args.copy_probe:
        src = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    forms = [f for f in args.forms.split(",") if f and f != "none"]
    if forms:
        line["forms"] = {}
    big32 = None
    if "fp32" in forms:
        line["forms"]["fp32"] = form_fp32(torch, dev, args.fp32_n, args.fp32_steps)
        big32 = line["forms"]["fp32"]["gaussian_pulse"]["value"]
    if "adjoint" in forms:
        line["forms"]["adjoint"] = form_adjoint(torch, dev, args.adj_n, args.adj_steps, ndir=args.adj_dirs)
    if "batch" in forms:
        line["forms"]["batch"] = form_batch(torch, dev, args.batch_count, args.batch_steps, big32, lite=args.batch_lite)
    if "fc" in forms:
        line["forms"]["fc"] = form_fc(torch, dev, args.fc_n, args.fc_steps)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        if args.cpu_sample_n:
            line["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.cpu_sample_steps)
        else:
            line["cpu_baseline"] = cpu_baseline(P.nx, args.cpu_sample_steps, P, s0)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
