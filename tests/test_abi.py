"""The C-ABI library builds, loads, and exports every entry point that
include/tsgls.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsgls.h")
LIB = os.path.join(ROOT, "paper_2311_09465_amd", "libtsgls.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tsgls_[a-z_A-Z0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("tsgls_create", "tsgls_set_dirichlet", "tsgls_set_neumann", "tsgls_residual",
                 "tsgls_linearize", "tsgls_jv", "tsgls_jacobi_diag", "tsgls_get_tau",
                 "tsgls_solve", "tsgls_last_error", "tsgls_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libtsgls.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_supported_K_and_argument_errors_without_gpu():
    lib = ctypes.CDLL(LIB)
    buf = (ctypes.c_int * 64)()
    n = lib.tsgls_supported_K(buf, 64)
    ks = [buf[i] for i in range(n)]
    assert {0, 1, 2, 3, 6}.issubset(ks)
    # null output handle and null mesh are rejected before any device call
    assert lib.tsgls_create(None, 0, None, 0, None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.tsgls_create(None, 4, None, 1, None, None, ctypes.byref(out)) == -1
    lib.tsgls_last_error.restype = ctypes.c_char_p
    assert lib.tsgls_last_error(None) == b"null context"


def test_extension_entry_points_reject_bad_arguments_without_gpu():
    """Batched solves, tracer mode, reduced basis and network validate their
    arguments before any device call."""
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.tsgls_solve_batch.argtypes = [P, P, ctypes.c_int, P, P, P, ctypes.c_int]
    assert lib.tsgls_solve_batch(None, None, -1, None, None, None, 0) == -1
    assert lib.tsgls_solve_batch(None, None, 0, None, None, None, 0) == 0     # empty batch
    assert lib.tsgls_solve_batch(None, None, 2, None, None, None, 0) == -1
    lib.tsgls_set_tracer.argtypes = [P, P, ctypes.c_double, ctypes.c_int]
    assert lib.tsgls_set_tracer(None, None, 1.0, 1) == -1
    lib.tsgls_set_segments.argtypes = [P, ctypes.c_int]
    assert lib.tsgls_set_segments(None, 2) == -1
    lib.tsgls_solve_segments.argtypes = [P, P, P, P, P]
    assert lib.tsgls_solve_segments(None, None, None, None, None) == -1
    lib.tsgls_jv_prec.argtypes = [P, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_int]
    assert lib.tsgls_jv_prec(None, None, None, 0, 0.0, 0) == -1
    lib.tsgls_rb_greedy.argtypes = [P, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int, P, P, P]
    assert lib.tsgls_rb_greedy(None, 4, 10, None, 2, None, None, None) == -1
    lib.tsgls_rb_project.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, ctypes.c_int64, P, P, P]
    assert lib.tsgls_rb_project(None, 2, 10, None, 1, None, None, None) == -1
    lib.tsgls_rb_expand.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, P, P, P]
    assert lib.tsgls_rb_expand(None, 2, 10, None, None, None, None) == -1
    lib.tsgls_mlp_create.argtypes = [ctypes.c_int] * 5 + [ctypes.c_uint64, P, P]
    out = ctypes.c_void_p()
    assert lib.tsgls_mlp_create(0, 8, 2, 3, 0, 1, None, ctypes.byref(out)) == -1
    assert lib.tsgls_mlp_create(4, 8, 2, 3, 7, 1, None, ctypes.byref(out)) == -1
    assert out.value is None
    lib.tsgls_mlp_last_error.restype = ctypes.c_char_p
    lib.tsgls_mlp_last_error.argtypes = [P]
    assert lib.tsgls_mlp_last_error(None) == b"null network"
