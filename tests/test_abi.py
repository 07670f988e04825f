"""The C-ABI library loads and exports every entry point the header declares,
and host-side validation works without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spc3d.h")
LIB = os.path.join(ROOT, "paper_2404_19638_amd", "libspc3d.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spc3d_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libspc3d.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("spc3d_plan_create_coo", "spc3d_gather", "spc3d_sddmm", "spc3d_spmm",
              "spc3d_scatter_reduce", "spc3d_row_softmax", "spc3d_row_softmax_bwd"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_validation(lib):
    sz = ctypes.c_size_t()
    f = lib.spc3d_plan_workspace_size
    f.argtypes = [ctypes.c_int64] * 5 + [ctypes.c_uint32, ctypes.POINTER(ctypes.c_size_t)]
    assert f(1000, 0, 100, 0, 100, 0, ctypes.byref(sz)) == 0 and sz.value > 0
    small = sz.value
    assert f(1000, 0, 100, 0, 100, 1, ctypes.byref(sz)) == 0 and sz.value > small  # CSC adds
    assert f(-1, 0, 100, 0, 100, 0, ctypes.byref(sz)) == 1          # negative nnz
    assert f(10, 5, 5, 0, 100, 0, ctypes.byref(sz)) == 1            # empty range
    assert f(10, 0, 100, 0, 100, 8, ctypes.byref(sz)) == 1          # unknown flag
    lib.spc3d_last_error.restype = ctypes.c_char_p
    assert b"flags" in lib.spc3d_last_error()
    q = lib.spc3d_plan_query
    q.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3
    R = ctypes.c_int64()
    assert q(None, ctypes.byref(R), None, None) == 6                 # bad handle
    forged = ctypes.create_string_buffer(256)
    assert q(ctypes.cast(forged, ctypes.c_void_p), ctypes.byref(R), None, None) == 6
    lib.spc3d_plan_destroy.argtypes = [ctypes.c_void_p]
    assert lib.spc3d_plan_destroy(ctypes.cast(forged, ctypes.c_void_p)) == 6
    lib.spc3d_status_string.restype = ctypes.c_char_p
    assert lib.spc3d_status_string(3) == b"workspace or buffer too small"
    assert lib.spc3d_version() >= 100
