"""ctypes binding of the C++ oracle (af_oracle.cpp).  Test infrastructure only.

All arrays are float64, C-contiguous; a state is (16, ny, nx) in the layout of
paper_2605_12915_amd.inputs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS = {0: "ok", 1: "acoustic_cfl", 2: "foot", 3: "nonphysical"}


def lib():
    global _LIB
    if _LIB is None:
        # AF_ORACLE_LIB selects another build of the same source (the sanitizer build)
        path = os.environ.get("AF_ORACLE_LIB") or os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path):
            from . import build
            build.build()
        L = ctypes.CDLL(path)
        D, I, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.orc_monomial_block.argtypes = [I, I, I, P]
        L.orc_wedge_apply.argtypes = [I, I, D, P, P]
        L.orc_wedge_apply.restype = I
        L.orc_centres.argtypes = [I, I, D, D, P, P]
        L.orc_increments.argtypes = [I, I, D, D, D, I, P, P]
        L.orc_increments.restype = D
        L.orc_feet.argtypes = [I, I, D, D, D, I, P, P, P]
        L.orc_step.argtypes = [I, I, D, D, D, I, I, P, P]
        L.orc_run.argtypes = [I, I, D, D, D, I, I, I, P, P]
        L.orc_step_jvp.argtypes = [I, I, D, D, D, I, I, P, P, P, P]
        L.orc_diagnostics.argtypes = [I, I, D, D, D, P, P]
        L.orc_num_threads_default.restype = I
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    return int(lib().orc_num_threads_default())


def monomial_block(a: int, b: int, quad_mask: int) -> np.ndarray:
    C = np.zeros(9)
    lib().orc_monomial_block(a, b, quad_mask, _p(C))
    return C.reshape(3, 3)


def wedge_apply(fam: int, w: int, r: float, f: np.ndarray) -> np.ndarray:
    """f: (3 vars (pi,u,v), 3 x-nodes, 3 y-nodes) -> (pi, u, v) contribution."""
    f = _c(f)
    out = np.zeros(3)
    st = lib().orc_wedge_apply(fam, w, float(r), _p(f), _p(out))
    if st:
        raise ValueError("bad wedge")
    return out


def centres(state, h, gamma):
    s = _c(state)
    _, ny, nx = s.shape
    out = np.zeros((4, ny, nx))
    lib().orc_centres(nx, ny, h, gamma, _p(s), _p(out))
    return out


def increments(state, h, gamma, tau, threads=None):
    s = _c(state)
    _, ny, nx = s.shape
    out = np.zeros((4, 3, ny, nx))
    rmax = lib().orc_increments(nx, ny, h, gamma, tau, threads or default_threads(), _p(s), _p(out))
    return out, rmax


def feet(state, h, gamma, tau, scheme=0):
    s = _c(state)
    _, ny, nx = s.shape
    ft = np.zeros((3, 2, ny, nx))
    pts = np.zeros((3, 4, ny, nx))
    st = lib().orc_feet(nx, ny, h, gamma, tau, scheme, _p(s), _p(ft), _p(pts))
    return ft, pts, st


def step(state, h, gamma, dt, scheme=0, threads=None, check=True):
    s = _c(state)
    _, ny, nx = s.shape
    out = np.zeros_like(s)
    st = lib().orc_step(nx, ny, h, gamma, dt, scheme, threads or default_threads(), _p(s), _p(out))
    if check and st:
        raise RuntimeError(f"oracle step failed: {STATUS.get(st, st)}")
    return out if not (not check and st) else (out, st)


def run(state, h, gamma, dt, nsteps, scheme=0, threads=None):
    s = _c(state)
    _, ny, nx = s.shape
    out = np.zeros_like(s)
    st = lib().orc_run(nx, ny, h, gamma, dt, scheme, threads or default_threads(), nsteps, _p(s), _p(out))
    if st:
        raise RuntimeError(f"oracle run failed: {STATUS.get(st, st)}")
    return out


def step_jvp(state, direction, h, gamma, dt, scheme=0, threads=None):
    """Complex-step: returns (step(state), J @ direction), both exact to round-off."""
    s = _c(state)
    d = _c(direction)
    _, ny, nx = s.shape
    out = np.zeros_like(s)
    jv = np.zeros_like(s)
    st = lib().orc_step_jvp(nx, ny, h, gamma, dt, scheme, threads or default_threads(),
                            _p(s), _p(d), _p(out), _p(jv))
    if st:
        raise RuntimeError(f"oracle jvp failed: {STATUS.get(st, st)}")
    return out, jv


def diagnostics(state, h, gamma, dt):
    s = _c(state)
    _, ny, nx = s.shape
    out = np.zeros(11)
    lib().orc_diagnostics(nx, ny, h, gamma, dt, _p(s), _p(out))
    keys = ["mass", "momx", "momy", "energy", "entropy", "min_rho", "min_p", "max_speed", "max_acoustic_r",
            "vorticity", "enstrophy"]
    return dict(zip(keys, out.tolist()))
