"""The algorithmic flop counts the benchmark reports are the ones the kernels'
arithmetic performs for one cell's own work, forward step and adjoint step (host
build of csrc/count_flops.cpp)."""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_12915_amd", "csrc")


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc missing")
def test_flop_count_current(tmp_path):
    from paper_2605_12915_amd import perf
    exe = str(tmp_path / "count_flops")
    subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-std=c++17", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
                    os.path.join(CSRC, "count_flops.cpp"), "-o", exe], check=True, capture_output=True)
    out = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    assert out["flops_per_cell_update"] == perf.ALGO_FLOPS_PER_CELL_F64
    assert out["sqrts"] == 4 and out["divs"] > 0
    # the adjoint's share per cell: its parts add up, and it re-forms the forward
    # intermediates (centre and increments) exactly once
    parts = ("adjoint_forward_intermediates", "adjoint_points", "adjoint_increments", "adjoint_centre")
    assert sum(out[k] for k in parts) == out["adjoint_flops_per_cell"] == perf.ALGO_FLOPS_PER_CELL_ADJ
    assert out["adjoint_forward_intermediates"] == (out["centre"] + out["increments_V"] + out["increments_Ev_Eh"]
                                                    + out["increments_C"])


def test_dominant_kernel_has_tracked_sources():
    """The kernel the benchmark reports has a source list, so stored counters are
    invalidated when its code changes (perf.stored_traffic)."""
    import re
    from paper_2605_12915_amd import perf
    src = open(os.path.join(ROOT, "paper_2605_12915_amd", "csrc", "af_api.hip")).read()
    names = re.findall(r'"(af::k_fused<double, af::PolAbs<double>, [^"]*, 0, [^"]*)"', src)
    assert names, "dominant FP64 kernel name not found"
    for n in names:
        assert perf.source_sha(n) is not None, n
