"""Benchmark of the RB-TAI Active Flux step on one MI355X.

Workload (N = 1): periodic 2048 x 2048 grid, FP64, background rho = 1, p = 1/1.4,
(u, v) = (0.5, 0.3) plus 16 seeded Fourier modes per primitive field (wavenumbers
up to 8, amplitude 1e-3), CFL 0.4.  Inputs are generated on the host, copied to HBM
before the timed region; K steps are timed between two device synchronisations.

Prints ONE JSON line (see the design doc for every field's definition).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)



def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=512)
    ap.add_argument("--cpu-sample-steps", type=int, default=6)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(n: int, steps: int):
    """The oracle as it stands, on the host cores, over a bounded sample of the same
    workload family (smaller grid, few steps)."""
    from oracle import ref
    from paper_2605_12915_amd import inputs as I
    P = I.fourier_modes(n)
    s = P.state()
    dt = P.dt_for_cfl(0.4)
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref.run(s, P.h, P.gamma, dt, steps, threads=threads)
    el = time.perf_counter() - t0
    return {"value": n * n * steps / el / 1e6, "unit": "Mcell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} Fourier-mode flow, {steps} steps, FP64, {threads} OpenMP threads, {el:.2f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2605_12915_amd import inputs as I
    from paper_2605_12915_amd.stepper import Stepper

    dev = torch.device("cuda:0")
    P = I.fourier_modes(args.n)
    s0 = P.state()
    dt = P.dt_for_cfl(0.4)
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev)
    x = torch.from_numpy(s0).to(dev)
    torch.cuda.synchronize()
    if args.warmup:
        st.step(x, dt, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(x, dt, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ncell = P.nx * P.ny
    value = ncell * args.steps / el / 1e6
    # dominant-kernel duration from HIP events on the library's stream
    tot_ms, ker_ms = st.time_steps(x, dt, 20)
    diag = st.diagnostics(x, dt)
    ok = bool(np.isfinite(diag["mass"]))
    from paper_2605_12915_amd import perf
    kname = st.dominant_kernel()
    flops = perf.ALGO_FLOPS_PER_CELL_F64 * ncell            # per launch of the step kernel
    achieved = flops / (ker_ms * 1e-3) / 1e12
    t_alu = flops / (perf.FP64_PEAK_TFLOPS * 1e12)
    t_hbm = perf.ALGO_BYTES_PER_CELL_F64 * ncell / (perf.HBM_PEAK_GBS * 1e9)
    tr = perf.stored_traffic(kname)
    line = {
        "metric": "Mcell-updates/s per AF step (FP64 vs FP32) at stated error; adjoint/forward ratio",
        "value": value, "unit": "Mcell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
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
                     "t_alu_ms": t_alu * 1e3, "t_hbm_ms": t_hbm * 1e3},
        "finite": ok,
    }
    if args.copy_probe:
        src = torch.empty(128 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_n, args.cpu_sample_steps)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
