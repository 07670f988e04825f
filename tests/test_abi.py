"""The C-ABI library loads and exports every entry point the header declares,
and host-side validation works without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spc3d.h")
# SPC3D_LIB names another build of the library (the host sanitizer build)
LIB = os.environ.get("SPC3D_LIB") or os.path.join(ROOT, "paper_2404_19638_amd", "libspc3d.so")


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
    lib.spc3d_plan_check.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.spc3d_plan_check(None, None) == 6                      # bad handle
    assert lib.spc3d_plan_check(ctypes.cast(forged, ctypes.c_void_p), None) == 6
    assert lib.spc3d_debug_bounds() == (1 if os.environ.get("SPC3D_DEBUG_BOUNDS", "0")
                                        not in ("", "0") else 0)


def test_variant_check_rules(lib):
    """spc3d_variant_check is host-only: the shape rules without a launch."""
    f = lib.spc3d_variant_check
    f.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.c_int, ctypes.c_int]
    SDDMM, SPMM, FUSED = 0, 1, 2
    F32, BF16 = 0, 1
    OK, INVALID, UNSUPPORTED = 0, 1, 4

    def var(lanes, items, wide=0, window=0):
        return lanes | (items << 4) | (wide << 8) | (0x200 if window else 0)

    for op in (SDDMM, SPMM, FUSED):
        assert f(op, 32, F32, -1) == OK and f(op, 128, BF16, -1) == OK
        assert f(op, 32, F32, 0) == INVALID            # 1 lane per entry is not a shape
        assert f(op, 32, F32, var(7, 0)) == INVALID
        assert f(op, 32, F32, var(3, 5)) == INVALID     # items beyond 1024 slots
        assert f(op, 32, F32, var(3, 0, 1, 1)) == INVALID   # wide and window together
        assert f(op, 32, F32, 0x400 | 3) == INVALID
        assert f(op, 0, F32, -1) == INVALID and f(op, 32, 7, -1) == INVALID
    assert f(3, 32, F32, -1) == INVALID
    # kz = 128 FP32 is 32 vectors: 2 lanes would need 16 per lane
    assert f(SDDMM, 128, F32, var(1, 0)) == UNSUPPORTED
    assert f(SDDMM, 128, F32, var(3, 0)) == OK
    # group-run SpMM needs >= 8 slots per group (16 with wide batches)
    assert f(SPMM, 32, F32, var(3, 0)) == OK            # 64 slots / 8 groups
    assert f(SPMM, 32, F32, var(2, 0)) == UNSUPPORTED   # 64 / 16 groups = 4
    assert f(SPMM, 32, F32, var(3, 0, 1)) == UNSUPPORTED
    assert f(SPMM, 32, F32, var(3, 1, 1)) == OK
    # the windowed family has no run-length rule but takes 2, 4 or 8 lanes
    assert f(SPMM, 32, F32, var(2, 0, 0, 1)) == OK
    assert f(FUSED, 32, F32, var(3, 4, 0, 1)) == OK
    assert f(SPMM, 32, F32, var(4, 0, 0, 1)) == UNSUPPORTED
    # SDDMM ignores the SpMM bits
    assert f(SDDMM, 32, F32, var(4, 0, 0, 1)) == OK


def test_host_validation_of_the_widening_entry_points(lib):
    """Argument checks that return before any device work."""
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    lo_ = lib.spc3d_lambda_owners
    lo_.argtypes = [i32, vp, vp, i64, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    assert lo_(0, None, None, 0, 10, None, None, None, None, None, None, 0, None) == 4
    assert lo_(65, None, None, 0, 10, None, None, None, None, None, None, 0, None) == 4
    ws = lib.spc3d_lambda_owners_workspace_size
    ws.argtypes = [i64, i64, ctypes.POINTER(sz)]
    b = sz()
    assert ws(5, 5, ctypes.byref(b)) == 1
    assert ws(0, 100, ctypes.byref(b)) == 0 and b.value >= 800
    g = lib.spc3d_plan_create_coo_grouped
    g.argtypes = [ctypes.POINTER(vp), i64, vp, vp, i64, i64, i64, i64, vp, i32, vp, i32,
                  ctypes.c_uint32, vp, sz, vp]
    h = vp()
    fake = ctypes.c_void_p(16)   # never dereferenced: the count check comes first
    assert g(ctypes.byref(h), 0, None, None, 0, 10, 0, 10, fake, 0, None, 0, 0, None, 0,
             None) == 1
    assert g(ctypes.byref(h), 0, None, None, 0, 10, 0, 10, fake, 5000, None, 0, 0, None, 0,
             None) == 1
    c = lib.spc3d_plan_create_csr
    c.argtypes = [ctypes.POINTER(vp), i64, vp, vp, i64, i64, i64, i64, ctypes.c_uint32, vp, sz,
                  vp]
    assert c(ctypes.byref(h), 0, None, None, 0, 10, 0, 10, 0, None, 0, None) == 1
    go = lib.spc3d_plan_group_offsets
    go.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(i32)]
    assert go(None, 0, None, None) == 6


def test_c_client_compiles_against_the_header_and_links():
    """A plain C program (gcc, C11, -Wall -Wextra) includes include/spc3d.h and
    links libspc3d.so: the boundary needs no C++ and no PyTorch."""
    import importlib.util
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location(
        "abi_client_build", os.path.join(here, "abi_client", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert os.path.exists(mod.build())


def test_size_limits_are_exact_and_overflow_safe():
    """The documented limits, checked on the host: id ranges of 1..2^31-2 ids,
    nnz up to 2^31-65; a range with hi <= lo, one id too wide, or spanning the
    whole int64 line (whose width overflows int64) is refused."""
    from paper_2404_19638_amd import spc3d as spc
    n = (1 << 31) - 2
    assert spc.plan_workspace_size(10, 1 << 40, (1 << 40) + n, 5 << 40, (5 << 40) + n) > 0
    assert spc.plan_workspace_size((1 << 31) - 65, 0, 10, 0, 10) > 0
    for args in [(10, 0, n + 1, 0, 10), (10, 0, 10, 7, n + 8), (10, 5, 5, 0, 10),
                 (10, 0, 10, 9, 3), (10, -(1 << 63), (1 << 63) - 1, 0, 10),
                 ((1 << 31) - 64, 0, 10, 0, 10), (-1, 0, 10, 0, 10)]:
        with pytest.raises(spc.Spc3dError) as ei:
            spc.plan_workspace_size(*args)
        assert ei.value.status == spc.ERR_INVALID_ARG, args
