"""Host build of the GPU's foot-centred exact point update (af_footcentred.h through
tests/fc_host.cpp) against the oracle (oracle/footcentred.py): the same feet, frozen
states and disk quadratures, computed by independent code (CPU only)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from oracle import footcentred as fc
from paper_2605_12915_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_12915_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def fc_host(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc missing")
    d = tmp_path_factory.mktemp("fc_host")
    exe = str(d / "fc_host")
    subprocess.run([HIPCC, "-std=c++17", "-O1", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
                    os.path.join(ROOT, "tests", "fc_host.cpp"), "-o", exe], check=True, capture_output=True,
                   timeout=900)

    def run(s, h, g, dt):
        _, ny, nx = s.shape
        fin, fout = str(d / "in.bin"), str(d / "out.bin")
        with open(fin, "wb") as f:
            f.write(struct.pack("<iiddd", nx, ny, h, g, dt))
            f.write(np.ascontiguousarray(s, np.float64).tobytes())
        subprocess.run([exe, fin, fout], check=True, timeout=600)
        b = open(fout, "rb").read()
        return struct.unpack("<i", b[:4])[0], np.frombuffer(b[4:], np.float64).reshape(2, 12, ny, nx)
    return run


@pytest.mark.parametrize("nx,ny,seed,vel,kmax", [(10, 8, 3, (0.25, -0.15), 3), (9, 11, 5, (-0.3, 0.2), 2)])
def test_host_point_values_equal_oracle(fc_host, nx, ny, seed, vel, kmax):
    P = I.random_smooth(nx, ny, seed=seed, amp=0.08, vel=vel, kmax=kmax)
    s0 = P.state()
    dt = P.dt_for_cfl(0.3)
    st, got = fc_host(s0, P.h, P.gamma, dt)
    assert st == 0
    want = np.stack([fc.point_values(s0, P.h, P.gamma, 0.5 * dt), fc.point_values(s0, P.h, P.gamma, dt)])
    scale = np.abs(want).max(axis=(2, 3), keepdims=True)
    assert (np.abs(got - want) / scale).max() <= 1e-13


def test_host_footprint_flag(fc_host):
    """A step long enough that |delta| + R reaches half a cell: the footprint bit (8)."""
    P = I.uniform(6, W=(1.0, 0.3, 0.0, 1.0))
    s0 = P.state()
    dt = 0.45 * P.h / (1.4 ** 0.5)
    st, _ = fc_host(s0, P.h, P.gamma, dt)
    assert st & 8
    with pytest.raises(fc.FootprintError):
        fc.point_values(s0, P.h, P.gamma, dt)
