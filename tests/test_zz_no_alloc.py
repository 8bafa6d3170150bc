"""Allocation-free adjoint entry point (af_step_adjoint_noalloc) against the context
form af_step_adjoint: same kernels, scratch in the library's static device array
instead of context memory.  Two calls in a row on one GPU, the second on a smaller
grid (the array keeps the first call's contents), both point updates; larger grids
are refused before any work."""
import ctypes

import numpy as np
import pytest

from paper_2605_12915_amd import inputs as I

pytestmark = pytest.mark.gpu

# FP64 atomic accumulation order differs between calls: agreement to round-off, not bits
TOL = 1e-12


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def _noalloc(torch, P, x, lam, dt, scheme, check=False):
    from paper_2605_12915_amd import _lib
    from paper_2605_12915_amd.stepper import state_struct
    cfg = _lib.AfConfig()
    cfg.nx, cfg.ny, cfg.h, cfg.gamma = P.nx, P.ny, P.h, P.gamma
    cfg.precision = _lib.AF_F64
    cfg.flags = (_lib.AF_SCHEME_RB if scheme == "rb" else 0) | (_lib.AF_CHECK if check else 0)
    out = torch.full_like(x, float("nan"))
    a, b, c = state_struct(x), state_struct(lam), state_struct(out)
    stream = torch.cuda.current_stream(x.device).cuda_stream
    code = _lib.lib().af_step_adjoint_noalloc(ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(a),
                                              ctypes.byref(b), ctypes.byref(c), float(dt))
    return code, out


def _ctx_adjoint(torch, dev, P, x, lam, dt, scheme):
    from paper_2605_12915_amd.stepper import Stepper
    st = Stepper(P.nx, P.ny, P.h, P.gamma, device=dev, scheme=scheme)
    want = st.adjoint(x, lam, dt)
    torch.cuda.synchronize()
    st.close()
    return want


def _rel(got, want):
    g, w = got.cpu().numpy(), want.cpu().numpy()
    return float((np.abs(g - w).max(axis=(1, 2)) / np.maximum(np.abs(w).max(axis=(1, 2)), 1e-300)).max())


@pytest.mark.parametrize("scheme", ["tai", "rb"])
def test_noalloc_matches_context_adjoint(torch_dev, scheme):
    torch, dev = torch_dev
    from paper_2605_12915_amd import _lib
    cases = [I.random_smooth(256, 256, seed=31, amp=0.1, vel=(0.3, -0.2)),    # the largest grid allowed
             I.random_smooth(45, 37, seed=32, amp=0.1, vel=(-0.25, 0.35))]    # then a smaller, ragged one
    for k, P in enumerate(cases):
        print(f"noalloc adjoint {scheme} call {k}: {P.nx}x{P.ny}", flush=True)
        s0 = P.state()
        dt = P.dt_for_cfl(0.4 if scheme == "tai" else 0.15)
        x = torch.from_numpy(s0).to(dev)
        lam = torch.from_numpy(np.random.default_rng(40 + k).normal(size=s0.shape)).to(dev)
        code, got = _noalloc(torch, P, x, lam, dt, scheme, check=(k == 1))
        assert code == _lib.AF_OK, _lib.lib().af_status_string(code)
        torch.cuda.synchronize()
        want = _ctx_adjoint(torch, dev, P, x, lam, dt, scheme)
        err = _rel(got, want)
        print(f"  max per-plane relative difference {err:.2e}", flush=True)
        assert np.isfinite(got.cpu().numpy()).all()
        assert err <= TOL


def test_noalloc_refuses_large_grid(torch_dev):
    torch, dev = torch_dev
    from paper_2605_12915_amd import _lib
    P = I.uniform(257, W=(1.0, 0.1, 0.0, 1.0), ny=256)          # 65792 cells > 65536
    s0 = P.state()
    x = torch.from_numpy(s0).to(dev)
    lam = torch.ones_like(x)
    code, out = _noalloc(torch, P, x, lam, 0.1 * P.h, "tai")
    assert code == _lib.AF_ERR_SCRATCH
    torch.cuda.synchronize()
    assert torch.isnan(out).all()                               # nothing was enqueued
