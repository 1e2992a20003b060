"""Host-side checks of the C-ABI library (no GPU): it loads, exports every declared
symbol, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hexpa.h")
LIB = os.path.join(ROOT, "paper_2603_09038_amd", "libhexpa.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_09038_amd.build import build
        build(quiet=True)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("pa_setup", "pa_apply", "pa_diag", "cg_solve", "pa_destroy", "pa_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    from paper_2603_09038_amd import hexpa
    assert sorted(hexpa.EXPORTS) == _declared()


def test_bad_arguments_are_rejected_without_a_device(lib):
    from paper_2603_09038_amd import hexpa
    h = ctypes.c_void_p()
    assert lib.pa_setup(None, 2, 4, None, 2, None, ctypes.byref(h)) == hexpa.PA_ERR_ARG
    assert lib.pa_setup(None, 2, 4, None, 2, None, None) == hexpa.PA_ERR_ARG
    lib.pa_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.pa_last_error()
    md = hexpa.MeshDesc()
    import numpy as np
    vert = np.zeros((8, 3))
    hexes = np.arange(8, dtype=np.int32)[None]
    md.nvert, md.vert_xyz, md.nelem, md.hex = 8, vert.ctypes.data, 1, hexes.ctypes.data
    md.nx = md.ny = md.nz = 1
    assert lib.pa_setup(ctypes.byref(md), 9, 10, None, 2, None, ctypes.byref(h)) == hexpa.PA_ERR_UNSUPPORTED
    assert lib.pa_setup(ctypes.byref(md), 2, 7, None, 2, None, ctypes.byref(h)) == hexpa.PA_ERR_UNSUPPORTED
    assert lib.pa_setup(ctypes.byref(md), 2, 4, None, 0, None, ctypes.byref(h)) == hexpa.PA_ERR_ARG
    md.nx = 2
    assert lib.pa_setup(ctypes.byref(md), 2, 4, None, 2, None, ctypes.byref(h)) == hexpa.PA_ERR_ARG
    md.nx = 1
    md.nelem = 0  # an empty mesh is rejected, not silently accepted
    assert lib.pa_setup(ctypes.byref(md), 2, 4, None, 2, None, ctypes.byref(h)) == hexpa.PA_ERR_ARG
    md.nelem, md.nvert = 1, 0
    assert lib.pa_setup(ctypes.byref(md), 2, 4, None, 2, None, ctypes.byref(h)) == hexpa.PA_ERR_ARG
    assert lib.pa_apply(None, None, None, None) == hexpa.PA_ERR_ARG
    assert lib.pa_diag(None, None, 0, None) == hexpa.PA_ERR_ARG
    assert lib.cg_solve(None, None, None, None, None, None) == hexpa.PA_ERR_ARG
    assert lib.pa_set_variant(None, 0) == hexpa.PA_ERR_ARG


def test_learned_preconditioner_rejects_bad_arguments_without_a_device(lib):
    from paper_2603_09038_amd import hexpa
    out = ctypes.c_void_p()
    o = hexpa._lp_opts()
    assert lib.pa_lp_create(None, ctypes.byref(o), ctypes.byref(out)) == hexpa.PA_ERR_ARG
    assert lib.pa_lp_create(None, ctypes.byref(o), None) == hexpa.PA_ERR_ARG
    assert lib.pa_lp_apply(None, None, None, None) == hexpa.PA_ERR_ARG
    assert lib.pa_lp_load(None, b"/nonexistent") == hexpa.PA_ERR_ARG
    assert lib.pa_lp_num_params() == 16 * 2 * 27 + 16 + 16 * 16 * 27 + 16 + 16 * 27 + 1
    bad = hexpa._lp_opts(coarse_iters=0)
    assert lib.pa_lp_configure(None, ctypes.byref(bad)) == hexpa.PA_ERR_ARG

