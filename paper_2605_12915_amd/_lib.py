"""ctypes binding of libaf.so (C ABI of include/af.h).  Argument marshalling only:
every step of the method runs in the HIP kernels of the library."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaf.so")

(AF_OK, AF_ERR_ARG, AF_ERR_HIP, AF_ERR_ACOUSTIC_CFL, AF_ERR_FOOT, AF_ERR_NONPHYSICAL, AF_ERR_UNSUPPORTED,
 AF_ERR_SCRATCH, AF_ERR_FOOTPRINT) = range(9)
AF_F64, AF_F32 = 0, 1
AF_CHECK, AF_SCHEME_RB, AF_SCHEME_FC = 1, 2, 4
SCHEME_FLAGS = {"tai": 0, "rb": AF_SCHEME_RB, "fc": AF_SCHEME_FC}

EXPORTED = [
    "af_init", "af_step", "af_step_out", "af_read_status", "af_step_adjoint", "af_diagnostics",
    "af_time_steps", "af_destroy", "af_status_string", "af_last_hip_error", "af_dominant_kernel",
    "af_init_batch", "af_step_batch", "af_batch_info", "af_reset_trajectory",
    "af_step_adjoint_noalloc",
]


class AfConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("h", ctypes.c_double), ("gamma", ctypes.c_double),
                ("precision", ctypes.c_int32), ("bg", ctypes.c_double * 4), ("flags", ctypes.c_int32)]


class AfState(ctypes.Structure):
    _fields_ = [("avg", ctypes.c_void_p * 4), ("V", ctypes.c_void_p * 4),
                ("EV", ctypes.c_void_p * 4), ("EH", ctypes.c_void_p * 4)]


class AfDiag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("mass", "momx", "momy", "energy", "entropy", "min_rho", "min_p", "max_speed", "max_acoustic_r",
                 "vorticity", "enstrophy")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class AfError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.af_status_string(code).decode()
        if code == AF_ERR_HIP:
            msg += f" (hipError {L.af_last_hip_error()})"
        super().__init__(f"{where}: {msg}")
        self.code = code


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libaf.so; raises if it has not been built (no fallback path exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2605_12915_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.af_init.argtypes = [ctypes.POINTER(AfConfig), P, ctypes.POINTER(P)]
        L.af_step.argtypes = [P, ctypes.POINTER(AfState), D, I32]
        L.af_step_out.argtypes = [P, ctypes.POINTER(AfState), ctypes.POINTER(AfState), D]
        L.af_read_status.argtypes = [P, ctypes.POINTER(I32)]
        L.af_step_adjoint.argtypes = [P, ctypes.POINTER(AfState), ctypes.POINTER(AfState), ctypes.POINTER(AfState), D]
        L.af_diagnostics.argtypes = [P, ctypes.POINTER(AfState), D, ctypes.POINTER(AfDiag)]
        L.af_time_steps.argtypes = [P, ctypes.POINTER(AfState), D, I32, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.af_reset_trajectory.argtypes = [P]
        L.af_step_adjoint_noalloc.argtypes = [ctypes.POINTER(AfConfig), P, ctypes.POINTER(AfState),
                                              ctypes.POINTER(AfState), ctypes.POINTER(AfState), D]
        L.af_destroy.argtypes = [P]
        L.af_destroy.restype = None
        L.af_status_string.argtypes = [I32]
        L.af_status_string.restype = ctypes.c_char_p
        L.af_last_hip_error.restype = I32
        L.af_init_batch.argtypes = [ctypes.POINTER(AfConfig), I32, P, ctypes.POINTER(P)]
        L.af_step_batch.argtypes = [P, ctypes.POINTER(AfState), ctypes.POINTER(D), I32]
        L.af_batch_info.argtypes = [P, ctypes.c_char_p, I32]
        L.af_batch_info.restype = I32
        L.af_dominant_kernel.argtypes = [P]
        L.af_dominant_kernel.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("af_destroy", "af_status_string", "af_last_hip_error", "af_dominant_kernel",
                            "af_batch_info"):
                getattr(L, name).restype = I32
        _LIB = L
    return _LIB


def check(code: int, where: str) -> None:
    if code != AF_OK:
        raise AfError(code, where)
