"""CPU checks of the C ABI: the library builds for gfx950, loads, and exports
every function include/bpmf.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bpmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bpmf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    import paper_1705_04159_amd as bp

    if not os.path.exists(bp.LIB_PATH):
        from paper_1705_04159_amd import build

        build.build()
    return bp.LIB_PATH


def test_header_declares_core_calls():
    names = _declared()
    for n in ["bpmf_create", "bpmf_sample_hyper", "bpmf_update_side", "bpmf_predict",
              "bpmf_run_sweeps", "bpmf_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    import paper_1705_04159_amd as bp

    assert sorted(bp.EXPORTS) == _declared()


def test_default_params_and_error_paths(libpath):
    """Host-only calls: defaults and argument validation fail before any GPU work."""
    import numpy as np

    import paper_1705_04159_amd as bp

    L = bp.lib()
    p = bp.Params()
    L.bpmf_default_params(ctypes.byref(p), 32)
    assert p.K == 32 and p.alpha == 2.0 and p.beta0 == 2.0 and p.nu0 == 32.0
    assert p.prec == bp.FP32 and p.center == 1 and p.foldin_S == 16
    ctx = ctypes.c_void_p()
    ptr = np.array([0, 1, 1], np.int64)
    col = np.array([5], np.int32)  # out of range for N = 3
    val = np.array([1.0], np.float32)
    rc = L.bpmf_create(2, 3, ptr.ctypes.data, col.ctypes.data, val.ctypes.data, None, None, None,
                       1, None, None, None, 0, ctypes.byref(p), ctypes.byref(ctx))
    assert rc == bp.E_RANGE
    assert b"out of range" in L.bpmf_last_error(None)
    p.K = 0
    rc = L.bpmf_create(2, 3, ptr.ctypes.data, col.ctypes.data, val.ctypes.data, None, None, None,
                       1, None, None, None, 0, ctypes.byref(p), ctypes.byref(ctx))
    assert rc == bp.E_INVAL
