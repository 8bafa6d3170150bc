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

Algorithmic work per cell of the adjoint step (FP64): 384 B (primal state read,
cotangent of the output read, cotangent of the input written) and the operation
count of one cell's share of the reverse step, counted the same way from the
adjoint kernels' own arithmetic (forward intermediates recomputed, transposed
point updates with their foot recomputation, transposed increments, transposed
centre recovery; scattered contributions count as additions).

MI355X peaks: HBM3E 8.0 TB/s; FP64 vector 78.6 TFLOP/s (256 CUs x 4 SIMDs x
16 lanes x 2 flops x 2.4 GHz); FP32 vector 157.3 TFLOP/s.
"""
from __future__ import annotations

import hashlib
import re
import json
import os

ALGO_FLOPS_PER_CELL_F64 = 4466
ALGO_BYTES_PER_CELL_F64 = 256
ALGO_FLOPS_PER_CELL_ADJ = 14297
ALGO_BYTES_PER_CELL_ADJ = 384
ALGO_BYTES_PER_CELL_F32 = 160      # 16 float planes each way + 4 compensation planes read and written
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# Files whose change invalidates a stored counter measurement of a kernel (its
# sources, and the build script that holds the compiler flags), relative to the package.
_STEP = ["csrc/af_fused.h", "csrc/af_tile.h", "csrc/af_kernels.h", "csrc/af_device.h", "csrc/af_blocks.h", "csrc/af_internal.h",
         "build.py"]
_ADJ = ["csrc/af_adjoint.hip", "csrc/af_adjoint.h", "csrc/af_kernels.h", "csrc/af_device.h", "csrc/af_blocks.h",
        "csrc/af_internal.h", "build.py"]
# the three kernels of one adjoint step (TAI point update)
ADJOINT_KERNELS = ["af::k_adj_fwd", "af::k_adj_points<0, 8, 8, 2>", "af::k_adj_incr"]
KERNEL_SOURCES = {
    "af::k_fused<double, af::PolAbs<double>, 31, 10, 512, 0, false, 1, 32, true>": ["csrc/af_fused.hip"] + _STEP,
    "af::k_fused<float, af::PolPert<float>, 31, 10, 512, 0, true, 4, 32, true>": ["csrc/af_fused_f32.hip"] + _STEP,
    "af::k_fused_batch_direct<31, 10, 512, 4, 0, 32>": ["csrc/af_batch.hip", "csrc/af_batch.h"] + _STEP,
    **{k: _ADJ for k in ADJOINT_KERNELS},
    "af::k_fc_points": ["csrc/af_f64.hip", "csrc/af_footcentred.h", "csrc/af_gauss.h", "csrc/af_kernels.h",
                        "csrc/af_device.h", "csrc/af_blocks.h", "csrc/af_internal.h", "build.py"],
}


def _code_of(path: str) -> bytes:
    """A source file without its comments and with whitespace runs collapsed, so that
    edits of comments alone do not mark stored counters as stale (C/C++ // and /* */
    comments; # comments in Python files)."""
    with open(path, encoding="utf-8") as fh:
        text = fh.read()
    if path.endswith(".py"):
        text = re.sub(r"(?m)^\s*#.*$", "", text)
    else:
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
    return " ".join(text.split()).encode()


def source_sha(kernel: str) -> str | None:
    """Hash of the code (comments stripped) of the files a kernel is built from."""
    files = KERNEL_SOURCES.get(kernel)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        h.update(_code_of(os.path.join(HERE, f)))
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


def stored_traffic_sum(kernels):
    """Counter figures of a kernel sequence (one launch of each), summed; None unless
    every kernel has a current record."""
    recs = [stored_traffic(k) for k in kernels]
    if not recs or any(r is None for r in recs):
        return None
    out = {"traffic_bytes_per_launch": sum(r["traffic_bytes_per_launch"] for r in recs)}
    if all(r.get("executed_fp64_flops_per_launch") for r in recs):
        out["executed_fp64_flops_per_launch"] = sum(r["executed_fp64_flops_per_launch"] for r in recs)
    return out
