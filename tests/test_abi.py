"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/af.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "af.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_2605_12915_amd import _lib
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "af_init" in names and "af_step" in names and "af_step_adjoint" in names and "af_diagnostics" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_header():
    from paper_2605_12915_amd import _lib
    assert set(declared_functions()) == set(_lib.EXPORTED)


def test_bad_config_rejected_on_host(L):
    from paper_2605_12915_amd import _lib
    cfg = _lib.AfConfig()
    cfg.nx, cfg.ny, cfg.h, cfg.gamma = 3, 8, 0.1, 1.4
    ctx = ctypes.c_void_p()
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfg.nx, cfg.h = 8, -1.0
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfg.h, cfg.gamma = 0.1, 1.0
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    assert L.af_init(None, None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    # beyond 2^31 cells (byte counts and launch sizes would overflow)
    cfg.gamma, cfg.nx, cfg.ny = 1.4, 65536, 32769
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfg.nx, cfg.ny = 2 ** 31 - 1, 2 ** 31 - 1
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    assert L.af_step(None, None, 0.1, 1) == _lib.AF_ERR_ARG
    assert L.af_diagnostics(None, None, 0.1, None) == _lib.AF_ERR_ARG


def test_status_strings(L):
    from paper_2605_12915_amd import _lib
    for code in range(_lib.AF_ERR_FOOTPRINT + 1):
        assert L.af_status_string(code) != b"unknown status"
    assert b"CFL" in L.af_status_string(_lib.AF_ERR_ACOUSTIC_CFL)
    assert b"footprint" in L.af_status_string(_lib.AF_ERR_FOOTPRINT)


def test_footcentred_config_rules_on_host(L):
    """AF_SCHEME_FC: FP64 single-grid only and not with AF_SCHEME_RB (refused by af_init
    before any device work)."""
    from paper_2605_12915_amd import _lib
    cfg = _lib.AfConfig()
    cfg.nx, cfg.ny, cfg.h, cfg.gamma, cfg.precision = 8, 8, 0.125, 1.4, _lib.AF_F64
    cfg.flags = _lib.AF_SCHEME_FC | _lib.AF_SCHEME_RB
    ctx = ctypes.c_void_p()
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfg.flags = _lib.AF_SCHEME_FC
    cfg.precision = _lib.AF_F32
    cfg.bg[0], cfg.bg[3] = 1.0, 1.0
    assert L.af_init(ctypes.byref(cfg), None, ctypes.byref(ctx)) == _lib.AF_ERR_UNSUPPORTED


def test_bad_batch_config_rejected_on_host(L):
    from paper_2605_12915_amd import _lib
    cfgs = (_lib.AfConfig * 2)()
    for c in cfgs:
        c.nx, c.ny, c.h, c.gamma, c.precision = 8, 8, 0.1, 1.4, _lib.AF_F32
        c.bg[0], c.bg[3] = 1.0, 1.0
    ctx = ctypes.c_void_p()
    assert L.af_init_batch(cfgs, 0, None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    assert L.af_init_batch(None, 2, None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfgs[1].precision = _lib.AF_F64
    assert L.af_init_batch(cfgs, 2, None, ctypes.byref(ctx)) == _lib.AF_ERR_UNSUPPORTED
    cfgs[1].precision = _lib.AF_F32
    cfgs[1].flags = _lib.AF_SCHEME_RB          # mixed point updates in one batch
    assert L.af_init_batch(cfgs, 2, None, ctypes.byref(ctx)) == _lib.AF_ERR_UNSUPPORTED
    cfgs[1].flags = 0
    cfgs[1].ny = 3
    assert L.af_init_batch(cfgs, 2, None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfgs[1].ny, cfgs[1].bg[0] = 8, 0.0
    assert L.af_init_batch(cfgs, 2, None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    cfgs[1].bg[0] = 1.0
    cfgs[0].nx = cfgs[0].ny = cfgs[1].nx = cfgs[1].ny = 40000    # 3.2e9 cells in all
    assert L.af_init_batch(cfgs, 2, None, ctypes.byref(ctx)) == _lib.AF_ERR_ARG
    assert L.af_step_batch(None, None, None, 1) == _lib.AF_ERR_ARG
    assert L.af_batch_info(None, None, 0) == -1
