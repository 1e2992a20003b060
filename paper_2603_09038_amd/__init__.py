"""hexpa: partial-assembly H1 mass/diffusion operators and CG solves on MI355X (gfx950).

The compute path is the HIP library ``libhexpa.so`` (C-ABI in ``include/hexpa.h``);
``paper_2603_09038_amd.hexpa`` is its ctypes binding.  Import that module to use the
library: it raises if the shared library is not built (there is no CPU fallback).
"""
import os

PACKAGE_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PACKAGE_DIR, "libhexpa.so")


def build(quiet=False):
    from .build import build as _build
    return _build(quiet=quiet)
