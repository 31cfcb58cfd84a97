"""The C-ABI library loads and exports every function include/cubics.h
declares; error handling works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cubics.h")
LIB = os.path.join(ROOT, "paper_1909_09213_amd", "libcubics.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(cubics_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("cubics_create", "cubics_destroy", "cubics_load", "cubics_free",
                 "cubics_solve", "cubics_solve_batch", "cubics_root", "cubics_last_error"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcubics.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcubics.so not built")
def test_null_arguments_are_rejected_without_gpu_work():
    lib = ctypes.CDLL(LIB)
    lib.cubics_last_error.restype = ctypes.c_char_p
    lib.cubics_load.restype = ctypes.c_int
    out = ctypes.c_void_p()
    rc = lib.cubics_load(None, 0, None, None, None, 0, None, None, None, None, None, None, None,
                         None, ctypes.byref(out))
    assert rc == -1 and out.value is None
    assert b"ctx" in lib.cubics_last_error()
    lib.cubics_solve.restype = ctypes.c_int
    assert lib.cubics_solve(None, 0, None, None) == -1
    lib.cubics_features.restype = ctypes.c_int
    assert lib.cubics_features(None, None, 0, None) == -1
    lib.cubics_lns.restype = ctypes.c_int
    assert lib.cubics_lns(None, 0, None, None, None, 0, None, None, None, None, None, None, None, None,
                          None, None, None, None) == -1
    lib.cubics_autotune.restype = ctypes.c_int
    assert lib.cubics_autotune(None, 0, 0, None, ctypes.c_int64(1), None, None, None, None) == -1
    lib.cubics_free(None)
    lib.cubics_destroy(None)
