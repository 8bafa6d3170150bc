"""Checked builds (CPU only).

* The oracle built with address and undefined-behaviour sanitizers, loaded in place of
  the plain build, runs the oracle's pins (step, acoustic operator, diagnostics): any
  read or write outside an array, signed overflow or other undefined behaviour aborts
  the run.
* The fused step's tile index arithmetic walked on the host (tests/tile_bounds.cpp):
  every work item of every phase, through the node-level functions the kernels call,
  with the LDS tile as an ordinary object and every array subscript checked against
  its extent, on ragged and tiny grids with feet beyond the window's reach.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_12915_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


def _runtime(name):
    out = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ missing")
def test_oracle_pins_under_sanitizers():
    from oracle import build
    lib = build.build(sanitize=True)
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes missing")
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0", AF_ORACLE_LIB=lib)
    code = (
        "import sys, pytest\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from oracle import ref\n"
        "assert ref.lib()._name.endswith('liborc_san.so'), ref.lib()._name\n"
        "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', '-m', 'not gpu and not slow',\n"
        f"  {os.path.join(ROOT, 'tests', 'test_oracle_step.py')!r},\n"
        f"  {os.path.join(ROOT, 'tests', 'test_oracle_acoustic.py')!r},\n"
        f"  {os.path.join(ROOT, 'tests', 'test_oracle_diagnostics.py')!r}]))\n")
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert " passed" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc missing")
def test_tile_walk_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tile_bounds")
    cmd = [HIPCC, "-std=c++17", "-O0", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "tile_bounds.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=900)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "all items in bounds" in r.stdout
