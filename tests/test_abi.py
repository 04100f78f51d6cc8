"""The C-ABI library loads and exports every symbol include/fvim.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvim.h")
LIB = os.path.join(ROOT, "paper_1811_11558_amd", "libfvim.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "for", "sizeof")))


def test_header_declares_the_north_star_calls():
    names = declared_functions()
    for n in ("mindlin_apply", "boussinesq_apply", "return_map", "contact_solve", "elastoplastic_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_create_rejects_bad_grids_before_touching_a_device():
    from paper_1811_11558_amd import binding as b
    lib = b.load_library()
    m = b._Material(1.0, 0.3, 0.01, 0.1)
    h = ctypes.c_void_p()
    for g in (b._Grid(30, 32, 8, 1, 1, 1), b._Grid(32, 32, 1, 1, 1, 1), b._Grid(32, 32, 8, 1, 0, 1),
              b._Grid(32, 32, 600, 1, 1, 1), b._Grid(2, 32, 8, 1, 1, 1)):
        rc = lib.fvim_create(ctypes.byref(g), ctypes.byref(m), 0, 0, None, ctypes.byref(h))
        assert rc == b.FVIM_EINVAL
        assert lib.fvim_last_error()
    g = b._Grid(32, 32, 8, 1, 1, 1)
    bad = b._Material(1.0, 0.5, 0.01, 0.1)
    assert lib.fvim_create(ctypes.byref(g), ctypes.byref(bad), 0, 0, None, ctypes.byref(h)) == b.FVIM_EINVAL
    assert lib.fvim_create(ctypes.byref(g), ctypes.byref(m), 7, 0, None, ctypes.byref(h)) == b.FVIM_EINVAL
    assert lib.fvim_footprint_bytes(ctypes.byref(g), 0, 0) > 0
    assert lib.fvim_footprint_bytes(ctypes.byref(b._Grid(30, 32, 8, 1, 1, 1)), 0, 0) == 0
