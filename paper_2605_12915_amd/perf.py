"""Performance model constants of the RB-TAI step (used by the benchmark).

Algorithmic work per cell-update (FP64 step):
  * bytes: the time-n state read once and the time-(n+1) state written once,
    16 planes x 8 B each way = 256 B;
  * flops: the operation count of one cell's own work (centre recovery, the four
    node increments for both durations, three targets' point updates for both
    durations, their time-Simpson fluxes, one x- and one y-edge flux and the
    average update), counted by running the kernels' arithmetic on the host with
    an operation-counting scalar (csrc/count_flops.cpp; a test keeps the figure
    current).  Halo recomputation of a tiled kernel is not algorithmic work.

MI355X peaks: HBM3E 8.0 TB/s; FP64 vector 78.6 TFLOP/s (256 CUs x 4 SIMDs x
16 lanes x 2 flops x 2.4 GHz); FP32 vector 157.3 TFLOP/s.
"""
from __future__ import annotations

import hashlib
import json
import os

ALGO_FLOPS_PER_CELL_F64 = 4462
ALGO_BYTES_PER_CELL_F64 = 256
ALGO_BYTES_PER_CELL_F32 = 160      # 16 float planes each way + 4 compensation planes read and written
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# Files whose change invalidates a stored counter measurement of a kernel (its
# sources, and the build script that holds the compiler flags), relative to the package.
KERNEL_SOURCES = {
    "af::k_fused<double, af::PolAbs<double>, 26, 12, 512, 0, false, 1>":
        ["csrc/af_fused.hip", "csrc/af_fused.h", "csrc/af_kernels.h", "csrc/af_device.h", "csrc/af_blocks.h",
         "csrc/af_internal.h", "build.py"],
}


def source_sha(kernel: str) -> str | None:
    files = KERNEL_SOURCES.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    rec = data.get(kernel)
    sha = source_sha(kernel)
    if not rec or sha is None or rec.get("source_sha") != sha:
        return None
    return rec
