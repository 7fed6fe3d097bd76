"""CPU checks of the C ABI: the library builds for gfx950, loads, and exports
every function the headers under include/ declare (no compute calls: no GPU here)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(bpmf_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


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


def test_params_layout_matches_header(tmp_path):
    """The binding's Params mirrors bpmf_params field by field (offsets and
    size from the C compiler on the header)."""
    import subprocess

    import paper_1705_04159_amd as bp

    names = [n for n, _ in bp.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"bpmf.h\"\nint main(void){\n"
                   + "".join('printf("%%zu\\n", offsetof(bpmf_params, %s));\n' % n for n in names)
                   + 'printf("%zu\\n", sizeof(bpmf_params));\nreturn 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [getattr(bp.Params, n).offset for n in names] + [ctypes.sizeof(bp.Params)]
    assert got == want


def test_reorder_flag_validated(libpath):
    """params.reorder defaults to 0 and values other than 0 and 1 are
    rejected before any GPU work."""
    import numpy as np

    import paper_1705_04159_amd as bp

    L = bp.lib()
    p = bp.Params()
    L.bpmf_default_params(ctypes.byref(p), 8)
    assert p.reorder == 0
    p.reorder = 2
    ctx = ctypes.c_void_p()
    ptr = np.array([0, 1, 1], np.int64)
    col = np.array([1], np.int32)
    val = np.array([1.0], np.float32)
    rc = L.bpmf_create(2, 3, ptr.ctypes.data, col.ctypes.data, val.ctypes.data, None, None, None,
                       1, None, None, None, 0, ctypes.byref(p), ctypes.byref(ctx))
    assert rc == bp.E_INVAL
    assert b"reorder" in L.bpmf_last_error(None)


def test_peak_argument_checks(libpath):
    """The measurement calls reject bad sizes on the host, before any GPU work."""
    import paper_1705_04159_amd as bp

    L = bp.lib()
    v = ctypes.c_double()
    assert L.bpmf_peak_triad(1000, 1, ctypes.byref(v)) == bp.E_INVAL  # under 1 MiB
    assert L.bpmf_peak_triad((1 << 20) + 8, 1, ctypes.byref(v)) == bp.E_INVAL  # not a multiple of 16
    assert L.bpmf_peak_triad(1 << 20, 0, ctypes.byref(v)) == bp.E_INVAL
    assert L.bpmf_peak_compute(4, 1, ctypes.byref(v)) == bp.E_INVAL
    assert L.bpmf_peak_compute(-1, 1, ctypes.byref(v)) == bp.E_INVAL
    assert L.bpmf_peak_gather(1 << 20, 24, 10, 1, ctypes.byref(v)) == bp.E_INVAL  # row not 16-B multiple
    assert L.bpmf_peak_gather(1 << 20, 2048, 10, 1, ctypes.byref(v)) == bp.E_INVAL  # row over 1 KiB
    assert L.bpmf_peak_gather(64, 128, 10, 1, ctypes.byref(v)) == bp.E_INVAL  # source under one row
    assert L.bpmf_peak_gather(1 << 20, 128, 0, 1, ctypes.byref(v)) == bp.E_INVAL
    assert L.bpmf_peak_gather(1 << 20, 128, 10, 1, None) == bp.E_INVAL
