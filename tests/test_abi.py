"""The C-ABI library loads and exports every entry point include/tmhip.h
declares (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tmhip.h")
LIB = os.path.join(ROOT, "paper_2107_09879_amd", "libtmhip.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libtmhip.so is not built (python -m paper_2107_09879_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("tm_create", "tm_set_geometry", "tm_set_spheres", "tm_plane_wave_rhs", "tm_solve",
              "tm_apply_operator", "tm_near_field", "tm_far_field", "tm_adjoint_solve",
              "tm_grad_radius", "tm_detector_vector"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_host_only_entry_points(lib):
    lib.tm_coeff_count.restype = ctypes.c_int
    assert [lib.tm_coeff_count(l) for l in (0, 1, 2, 3, 4, 5, 6, 7)] == [0, 6, 16, 30, 48, 70, 96, 0]
    lib.tm_abi_version.restype = ctypes.c_int
    assert lib.tm_abi_version() == 1
    lib.tm_status_string.restype = ctypes.c_char_p
    assert lib.tm_status_string(0) == b"ok"
    assert lib.tm_status_string(-2) == b"enclosing spheres overlap"

    class Opts(ctypes.Structure):
        _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                    ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int)]

    o = Opts()
    lib.tm_default_opts(ctypes.byref(o))
    assert (o.tol, o.restart, o.precision, o.use_x0) == (1e-8, 50, 0, 0)
    # a null context is rejected, not dereferenced
    lib.tm_destroy(None)
    assert lib.tm_set_geometry(None, 1, None, ctypes.c_double(1.0), 1) == -1
    assert lib.tm_set_batch_autotune(None, 1) == -1
    pf, it = ctypes.c_int(), ctypes.c_int()
    assert lib.tm_get_batch_config(None, 1, ctypes.byref(pf), ctypes.byref(it)) == -1


def test_library_is_gfx950_code():
    out = open(LIB, "rb").read()
    assert b"gfx950" in out
