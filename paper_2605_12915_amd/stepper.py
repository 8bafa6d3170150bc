"""PyTorch-facing wrapper of the C ABI.  Torch provides device memory and the stream
only; the step, its adjoint and the diagnostics run in libaf.so's HIP kernels.

A state is a (16, ny, nx) tensor on the GPU in the plane layout of include/af.h:
[avg(rho, rho u, rho v, E), V(rho,u,v,p), EV(...), EH(...)], x fastest.
"""
from __future__ import annotations

import ctypes
import weakref
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import AF_CHECK, AF_F32, AF_F64, AF_SCHEME_RB, SCHEME_FLAGS, AfConfig, AfDiag, AfState, check


def state_struct(t: torch.Tensor) -> AfState:
    if t.dim() != 3 or t.shape[0] != 16 or not t.is_contiguous():
        raise ValueError("state must be a contiguous (16, ny, nx) tensor")
    if not t.is_cuda:
        raise ValueError("state must live on the GPU")
    s = AfState()
    base = t.data_ptr()
    stride = t.stride(0) * t.element_size()
    for k in range(4):
        s.avg[k] = base + k * stride
        s.V[k] = base + (4 + k) * stride
        s.EV[k] = base + (8 + k) * stride
        s.EH[k] = base + (12 + k) * stride
    return s


class Stepper:
    """One grid (nx, ny, h, gamma) bound to a HIP stream."""

    def __init__(self, nx: int, ny: int, h: float, gamma: float = 1.4, precision: str = "f64",
                 scheme: str = "tai", check_errors: bool = False, bg: Sequence[float] = (1.0, 0.0, 0.0, 1.0),
                 x0: float = 0.0, y0: float = 0.0, stream: Optional[torch.cuda.Stream] = None,
                 device: Optional[torch.device] = None):
        L = _lib.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg = AfConfig()
        cfg.nx, cfg.ny, cfg.x0, cfg.y0, cfg.h, cfg.gamma = nx, ny, x0, y0, h, gamma
        cfg.precision = AF_F64 if precision == "f64" else AF_F32
        for k in range(4):
            cfg.bg[k] = float(bg[k])
        if scheme not in SCHEME_FLAGS:
            raise ValueError(f"scheme must be one of {sorted(SCHEME_FLAGS)}")
        cfg.flags = (AF_CHECK if check_errors else 0) | SCHEME_FLAGS[scheme]
        self.cfg = cfg
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self._last_out = None      # FP32: the tensor holding the output the compensation belongs to
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.af_init(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx)),
                  "af_init")

    def close(self):
        if self._ctx and self._ctx.value:
            _lib.lib().af_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_state(self, t: torch.Tensor):
        if t.dtype != self.dtype or tuple(t.shape) != (16, self.cfg.ny, self.cfg.nx):
            raise ValueError(f"expected a (16, {self.cfg.ny}, {self.cfg.nx}) {self.dtype} tensor")
        if t.device != self.device:
            raise ValueError("state on the wrong device")

    def _follow(self, state: torch.Tensor, out: torch.Tensor):
        """FP32: the library continues the compensation when the input buffer is the
        previous output's; a different tensor at a reused address starts afresh."""
        if self.dtype != torch.float32:
            return
        last = self._last_out() if self._last_out is not None else None
        if last is not state:
            check(_lib.lib().af_reset_trajectory(self._ctx), "af_reset_trajectory")
        self._last_out = weakref.ref(out)

    def step(self, state: torch.Tensor, dt: float, nsteps: int = 1) -> torch.Tensor:
        """Advance in place; returns `state`."""
        self._check_state(state)
        s = state_struct(state)
        self._follow(state, state)
        check(_lib.lib().af_step(self._ctx, ctypes.byref(s), float(dt), int(nsteps)), "af_step")
        return state

    def step_out(self, state: torch.Tensor, dt: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._check_state(state)
        out = torch.empty_like(state) if out is None else out
        self._check_state(out)
        a, b = state_struct(state), state_struct(out)
        self._follow(state, out)
        check(_lib.lib().af_step_out(self._ctx, ctypes.byref(a), ctypes.byref(b), float(dt)), "af_step_out")
        return out

    def read_status(self) -> int:
        st = ctypes.c_int32()
        check(_lib.lib().af_read_status(self._ctx, ctypes.byref(st)), "af_read_status")
        return st.value

    def adjoint(self, primal: torch.Tensor, cot_next: torch.Tensor, dt: float,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
        for t in (primal, cot_next):
            self._check_state(t)
        out = torch.empty_like(primal) if out is None else out
        a, b, c = state_struct(primal), state_struct(cot_next), state_struct(out)
        check(_lib.lib().af_step_adjoint(self._ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), float(dt)),
              "af_step_adjoint")
        return out

    def diagnostics(self, state: torch.Tensor, dt: float = 0.0) -> dict:
        self._check_state(state)
        s = state_struct(state)
        d = AfDiag()
        check(_lib.lib().af_diagnostics(self._ctx, ctypes.byref(s), float(dt), ctypes.byref(d)), "af_diagnostics")
        return d.as_dict()

    def time_steps(self, state: torch.Tensor, dt: float, nsteps: int):
        self._check_state(state)
        s = state_struct(state)
        tot, ker = ctypes.c_double(), ctypes.c_double()
        check(_lib.lib().af_time_steps(self._ctx, ctypes.byref(s), float(dt), int(nsteps), ctypes.byref(tot),
                                       ctypes.byref(ker)), "af_time_steps")
        return tot.value, ker.value

    def dominant_kernel(self) -> str:
        return _lib.lib().af_dominant_kernel(self._ctx).decode()


class Batch:
    """Batching form: many FP32 perturbation grids (uneven sizes, each with its own h,
    gamma, background and dt) stepped together, one launch per step over all grids
    (tile shape and grid mode, persistent or one workgroup per tile, chosen by the
    library's autotuner), the nsteps launches replayed from a hipGraph (af_init_batch /
    af_step_batch)."""

    def __init__(self, grids: Sequence[dict], check_errors: bool = False, scheme: str = "tai",
                 stream: Optional[torch.cuda.Stream] = None, device: Optional[torch.device] = None):
        """grids: one dict per instance with keys nx, ny, h and optional gamma (1.4),
        bg ((1, 0, 0, 1)), x0, y0.  scheme: "tai" or "rb", for every grid."""
        L = _lib.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = len(grids)
        cfgs = (AfConfig * n)()
        for q, g in enumerate(grids):
            c = cfgs[q]
            c.nx, c.ny, c.h = int(g["nx"]), int(g["ny"]), float(g["h"])
            c.gamma = float(g.get("gamma", 1.4))
            c.x0, c.y0 = float(g.get("x0", 0.0)), float(g.get("y0", 0.0))
            c.precision = AF_F32
            bg = g.get("bg", (1.0, 0.0, 0.0, 1.0))
            for k in range(4):
                c.bg[k] = float(bg[k])
            c.flags = (AF_CHECK if check_errors else 0) | (AF_SCHEME_RB if scheme == "rb" else 0)
        self.cfgs = cfgs
        self.n = n
        self._last = None          # (weakrefs, data pointers) of the previous call's tensors
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.af_init_batch(cfgs, n, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx)),
                  "af_init_batch")

    def close(self):
        if self._ctx and self._ctx.value:
            _lib.lib().af_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, states: Sequence[torch.Tensor], dts: Sequence[float], nsteps: int = 1):
        """Advance every states[q] (float32 (16, ny_q, nx_q) perturbation tensors) in place."""
        if len(states) != self.n or len(dts) != self.n:
            raise ValueError(f"expected {self.n} states and dts")
        arr = (AfState * self.n)()
        for q, t in enumerate(states):
            c = self.cfgs[q]
            if t.dtype != torch.float32 or tuple(t.shape) != (16, c.ny, c.nx) or t.device != self.device:
                raise ValueError(f"instance {q}: expected a (16, {c.ny}, {c.nx}) float32 tensor on {self.device}")
            arr[q] = state_struct(t)
        d = (ctypes.c_double * self.n)(*[float(x) for x in dts])
        # a new tensor at a buffer address the previous call used would continue the old
        # compensation in the library (which tracks addresses): start afresh then
        if self._last is not None:
            refs, ptrs = self._last
            if any(r() is not t and t.data_ptr() == p for r, p, t in zip(refs, ptrs, states)):
                check(_lib.lib().af_reset_trajectory(self._ctx), "af_reset_trajectory")
        self._last = ([weakref.ref(t) for t in states], [t.data_ptr() for t in states])
        check(_lib.lib().af_step_batch(self._ctx, arr, d, int(nsteps)), "af_step_batch")
        return states

    def read_status(self) -> int:
        """Read and clear the batch's device status flag (synchronises the stream)."""
        st = ctypes.c_int32()
        check(_lib.lib().af_read_status(self._ctx, ctypes.byref(st)), "af_read_status")
        return st.value

    def info(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(8192)
        n = _lib.lib().af_batch_info(self._ctx, buf, len(buf))
        if n < 0:
            raise RuntimeError("af_batch_info failed")
        return json.loads(buf.value.decode())

    def dominant_kernel(self) -> str:
        return _lib.lib().af_dominant_kernel(self._ctx).decode()


def background_cons(bg, gamma):
    r, u, v, p = (float(x) for x in bg)
    return (r, r * u, r * v, p / (gamma - 1.0) + 0.5 * r * (u * u + v * v))


def to_perturbation(state, bg, gamma: float):
    """Absolute FP64 state (16, ny, nx) -> FP32 perturbation state about bg (host numpy):
    averages minus U(bg), point values minus bg.  Representation change only."""
    import numpy as np
    s = np.asarray(state, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.float32)
    Ub = background_cons(bg, gamma)
    for k in range(4):
        out[k] = s[k] - Ub[k]
        for f in range(3):
            out[4 + 4 * f + k] = s[4 + 4 * f + k] - float(bg[k])
    return out


def from_perturbation(state32, bg, gamma: float):
    """Inverse of to_perturbation, evaluated in FP64."""
    import numpy as np
    s = np.asarray(state32, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.float64)
    Ub = background_cons(bg, gamma)
    for k in range(4):
        out[k] = s[k] + Ub[k]
        for f in range(3):
            out[4 + 4 * f + k] = s[4 + 4 * f + k] + float(bg[k])
    return out
