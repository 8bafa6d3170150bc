"""Host build of the diagnostics' logarithm (csrc/af_math.h through tests/log_host.cpp):
within 2 ulp of the host's log over every binade, both sides of 1, the subnormals and
seeded random arguments (CPU only)."""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_12915_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


def test_log_pos_within_two_ulp(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc missing")
    exe = str(tmp_path / "log_host")
    subprocess.run([HIPCC, "-std=c++17", "-O1", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
                    os.path.join(ROOT, "tests", "log_host.cpp"), "-o", exe], check=True, capture_output=True,
                   timeout=900)
    out = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True, timeout=300).stdout)
    assert out["count"] > 10_000_000
    assert out["max_ulp"] <= 2, out
