"""Python binding of the spc3d C ABI (``include/spc3d.h``).

Argument marshalling only: every function forwards to the C entry point of
the same name (without the ``spc3d_`` prefix); PyTorch provides device memory
(tensors) and the HIP stream (``torch.cuda.current_stream()``).  There is no
fallback: if ``libspc3d.so`` is missing or a call fails, an exception is
raised.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspc3d.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_RANGE, ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_HIP, ERR_BAD_HANDLE = range(7)
F32, BF16 = 0, 1
ROWS, COLS = 0, 1
OVERWRITE, ACCUMULATE = 0, 1
BUILD_CSC = 1
CALLER_TO_SLOT, SLOT_TO_CALLER, SLOT_TO_COLUMN, COLUMN_TO_SLOT = 0, 1, 2, 3
OP_SDDMM, OP_SPMM, OP_SDDMM_SPMM = 0, 1, 2
NFEAT = 23
FEATURES_BUFFER_BYTES = 256
STATIC_SCRATCH_BYTES = 16 << 20


VARIANT_WINDOW = 0x200


def variant(lg_lanes: int, lg_items: int, wide: int = 0, window: int = 0) -> int:
    """SPC3D_VARIANT: 2^lg_lanes lanes per nonzero, 64 * 2^lg_items slots per work item;
    wide=1 gathers up to 16 rows per batch in SpMM (8 otherwise); window=1 picks the
    windowed SpMM family (SPC3D_VARIANT_WINDOW)."""
    return lg_lanes | (lg_items << 4) | (wide << 8) | (VARIANT_WINDOW if window else 0)


class Spc3dError(RuntimeError):
    def __init__(self, status: int, func: str, detail: str):
        super().__init__(f"{func} failed with status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    """Load libspc3d.so (built in-tree by ``build.py``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2404_19638_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u32, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sigs = {
        "spc3d_plan_workspace_size": [i64, i64, i64, i64, i64, u32, P(sz)],
        "spc3d_plan_create_coo": [P(vp), i64, vp, vp, i64, i64, i64, i64, u32, vp, sz, vp],
        "spc3d_plan_create_csr": [P(vp), i64, vp, vp, i64, i64, i64, i64, u32, vp, sz, vp],
        "spc3d_plan_create_coo_grouped": [P(vp), i64, vp, vp, i64, i64, i64, i64, vp, i32, vp,
                                          i32, u32, vp, sz, vp],
        "spc3d_plan_group_offsets": [vp, ctypes.c_int, P(vp), P(i32)],
        "spc3d_plan_query": [vp, P(i64), P(i64), P(i64)],
        "spc3d_plan_maps": [vp, vp],
        "spc3d_plan_destroy": [vp],
        "spc3d_plan_check": [vp, vp],
        "spc3d_gather": [vp, ctypes.c_int, vp, ctypes.c_int, i64, i32, i32, vp, ctypes.c_int, vp],
        "spc3d_sddmm": [vp, vp, vp, vp, ctypes.c_int, i32, vp, ctypes.c_int, ctypes.c_int, vp],
        "spc3d_spmm_buffer_size": [vp, ctypes.c_int, i32, ctypes.c_int, P(sz)],
        "spc3d_spmm": [vp, ctypes.c_int, vp, vp, ctypes.c_int, i32, vp, ctypes.c_int, ctypes.c_int,
                       vp, sz, vp],
        "spc3d_sddmm_spmm": [vp, vp, vp, vp, ctypes.c_int, i32, vp, vp, ctypes.c_int,
                             ctypes.c_int, vp, sz, vp],
        "spc3d_sddmm_spmm_scatter": [vp, vp, vp, vp, ctypes.c_int, i32, vp, ctypes.c_int, vp,
                                     i64, i32, ctypes.c_int, vp, sz, vp],
        "spc3d_sddmm_spmm_static": [vp, vp, vp, vp, ctypes.c_int, i32, vp, vp, ctypes.c_int,
                                    ctypes.c_int, vp],
        "spc3d_scatter_reduce": [vp, ctypes.c_int, vp, i32, vp, i64, i32, vp],
        "spc3d_permute_values": [vp, ctypes.c_int, vp, vp, vp],
        "spc3d_row_softmax_buffer_size": [vp, P(sz)],
        "spc3d_row_softmax": [vp, vp, vp, vp, sz, vp],
        "spc3d_row_softmax_bwd": [vp, vp, vp, vp, vp, sz, vp],
        "spc3d_mul_values": [vp, vp, vp, vp, vp],
        "spc3d_row_softmax_apply": [vp, vp, vp, vp, vp],
        "spc3d_lambda_owners_workspace_size": [i64, i64, P(sz)],
        "spc3d_lambda_owners": [i32, vp, vp, i64, i64, vp, vp, vp, vp, vp, vp, sz, vp],
        "spc3d_attention_fwd_buffer_size": [vp, i32, ctypes.c_int, ctypes.c_int, P(sz)],
        "spc3d_attention_fwd": [vp, vp, vp, vp, ctypes.c_int, i32, vp, vp, ctypes.c_int, vp, sz,
                                vp],
        "spc3d_variant_check": [ctypes.c_int, i32, ctypes.c_int, ctypes.c_int],
        "spc3d_plan_features": [vp, ctypes.c_int, i32, ctypes.c_int, vp, vp, sz, vp],
        "spc3d_mlp_linear_fwd": [ctypes.c_int] * 3 + [vp] * 4 + [ctypes.c_int, vp],
        "spc3d_mlp_linear_bwd_buffer_size": [ctypes.c_int] * 3 + [P(sz)],
        "spc3d_mlp_linear_bwd": [ctypes.c_int] * 3 + [vp] * 4 + [ctypes.c_int] + [vp] * 4
                                + [sz, vp],
        "spc3d_mlp_mse": [i64, vp, vp, vp, vp, vp, vp],
        "spc3d_mlp_adam": [i64, vp, vp, vp, vp] + [ctypes.c_float] * 4 + [ctypes.c_int, vp],
        "spc3d_mlp_masked_argmin": [ctypes.c_int, ctypes.c_int, vp, vp, i32, ctypes.c_float, vp,
                                    vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.spc3d_status_string.argtypes = [ctypes.c_int]
    L.spc3d_status_string.restype = ctypes.c_char_p
    L.spc3d_last_error.argtypes = []
    L.spc3d_last_error.restype = ctypes.c_char_p
    L.spc3d_version.argtypes = []
    L.spc3d_version.restype = ctypes.c_int
    L.spc3d_debug_bounds.argtypes = []
    L.spc3d_debug_bounds.restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int, func: str):
    if status != OK:
        raise Spc3dError(status, func, lib().spc3d_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(cond: bool, msg: str):
    """Host-side shape check before a launch (the C ABI cannot see tensor sizes)."""
    if not cond:
        raise ValueError(msg)


def _rows_of(t: torch.Tensor, kz: int) -> bool:
    """A packed operand is read as rows of kz values: a 2-D tensor must have
    exactly kz columns (a wider one would be read with the wrong stride)."""
    return t.dim() != 2 or t.shape[1] == kz


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype {t.dtype}")


class _Maps(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("gmap_r", "gmap_c", "lmap_r", "lmap_c", "rowptr",
                                                "colidx", "perm", "colptr", "rowidx_t", "slot_t")]


class Plan:
    """A localized block living in a caller-owned workspace tensor."""

    def __init__(self, handle, ws: torch.Tensor, row_range, col_range, flags):
        self.handle = handle
        self.ws = ws
        self.row_range = tuple(int(x) for x in row_range)
        self.col_range = tuple(int(x) for x in col_range)
        self.flags = flags
        R, C, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().spc3d_plan_query(handle, ctypes.byref(R), ctypes.byref(C), ctypes.byref(nnz)),
               "spc3d_plan_query")
        self.R, self.C, self.nnz = R.value, C.value, nnz.value
        self._bufs = {}

    def _view(self, addr, n, dtype):
        if addr is None or n == 0:
            return torch.empty(0, dtype=dtype, device=self.ws.device)
        off = addr - self.ws.data_ptr()
        nbytes = n * torch.empty(0, dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype)

    def maps(self) -> dict:
        """Device views of gmap/lmap/rowptr/colidx/perm (and the CSC arrays)."""
        m = _Maps()
        _check(lib().spc3d_plan_maps(self.handle, ctypes.byref(m)), "spc3d_plan_maps")
        rr = self.row_range[1] - self.row_range[0]
        cr = self.col_range[1] - self.col_range[0]
        out = dict(gmap_r=self._view(m.gmap_r, self.R, torch.int64),
                   gmap_c=self._view(m.gmap_c, self.C, torch.int64),
                   lmap_r=self._view(m.lmap_r, rr, torch.int32),
                   lmap_c=self._view(m.lmap_c, cr, torch.int32),
                   rowptr=self._view(m.rowptr, self.R + 1, torch.int32),
                   colidx=self._view(m.colidx, self.nnz, torch.int32),
                   perm=self._view(m.perm, self.nnz, torch.int32))
        if m.colptr:
            out.update(colptr=self._view(m.colptr, self.C + 1, torch.int32),
                       rowidx_t=self._view(m.rowidx_t, self.nnz, torch.int32),
                       slot_t=self._view(m.slot_t, self.nnz, torch.int32))
        return out

    def group_offsets(self, axis: int) -> torch.Tensor:
        """Device view of the ngroups + 1 first local ids of a grouped axis."""
        d = ctypes.c_void_p()
        ng = ctypes.c_int32()
        _check(lib().spc3d_plan_group_offsets(self.handle, axis, ctypes.byref(d), ctypes.byref(ng)),
               "spc3d_plan_group_offsets")
        return self._view(d.value, ng.value + 1, torch.int32)

    def buffer(self, key, nbytes):
        """Cached 256-byte aligned scratch tensor (torch allocations are aligned).
        One per plan and key: calls on one plan issued concurrently from
        several streams must each pass their own ``buf``."""
        b = self._bufs.get(key)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.ws.device)
            self._bufs[key] = b
        return b

    def __del__(self):
        try:
            if self.handle is not None and _lib is not None:
                _lib.spc3d_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


# --------------------------------------------------------------------- setup

def plan_workspace_size(nnz, row_lo, row_hi, col_lo, col_hi, flags=0) -> int:
    b = ctypes.c_size_t()
    _check(lib().spc3d_plan_workspace_size(nnz, row_lo, row_hi, col_lo, col_hi, flags,
                                           ctypes.byref(b)), "spc3d_plan_workspace_size")
    return b.value


def plan_create_coo(row_gid: torch.Tensor, col_gid: torch.Tensor, row_range, col_range,
                    flags: int = 0, ws: torch.Tensor | None = None, stream=None,
                    group_r: torch.Tensor | None = None, ngroups_r: int = 0,
                    group_c: torch.Tensor | None = None, ngroups_c: int = 0) -> Plan:
    """Localize a COO block of int64 global ids (device tensors).  Synchronizes.

    With group_r (int32 device tensor, one key per id of the row range, keys
    in [0, ngroups_r)) local rows are ordered by (key, global id) -- the
    owner-grouped order (spc3d_plan_create_coo_grouped); likewise group_c."""
    assert row_gid.dtype == torch.int64 and col_gid.dtype == torch.int64
    assert row_gid.is_contiguous() and col_gid.is_contiguous()
    for g, rng in ((group_r, row_range), (group_c, col_range)):
        if g is not None:
            _need(g.dtype == torch.int32 and g.is_contiguous() and g.numel() >= rng[1] - rng[0],
                  "group keys: int32, one per id of the range")
    nnz = row_gid.numel()
    need = plan_workspace_size(nnz, row_range[0], row_range[1], col_range[0], col_range[1], flags)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=row_gid.device)
    h = ctypes.c_void_p()
    if group_r is None and group_c is None:
        _check(lib().spc3d_plan_create_coo(ctypes.byref(h), nnz, _ptr(row_gid), _ptr(col_gid),
                                           row_range[0], row_range[1], col_range[0],
                                           col_range[1], flags, _ptr(ws), ws.numel(),
                                           _stream(stream)), "spc3d_plan_create_coo")
    else:
        _check(lib().spc3d_plan_create_coo_grouped(
            ctypes.byref(h), nnz, _ptr(row_gid), _ptr(col_gid), row_range[0], row_range[1],
            col_range[0], col_range[1], _ptr(group_r), ngroups_r, _ptr(group_c), ngroups_c,
            flags, _ptr(ws), ws.numel(), _stream(stream)), "spc3d_plan_create_coo_grouped")
    return Plan(h, ws, row_range, col_range, flags)


def plan_create_csr(rowptr: torch.Tensor, col_gid: torch.Tensor, row_range, col_range,
                    flags: int = 0, ws: torch.Tensor | None = None, stream=None) -> Plan:
    """Localize a block given in CSR over its global row range: int64 rowptr
    (one entry per row of the range, plus one) and int64 global column ids in
    row order (device tensors).  Synchronizes."""
    assert rowptr.dtype == torch.int64 and col_gid.dtype == torch.int64
    assert rowptr.is_contiguous() and col_gid.is_contiguous()
    _need(rowptr.numel() == row_range[1] - row_range[0] + 1,
          "rowptr needs one entry per row of the range, plus one")
    nnz = col_gid.numel()
    need = plan_workspace_size(nnz, row_range[0], row_range[1], col_range[0], col_range[1], flags)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=col_gid.device)
    h = ctypes.c_void_p()
    _check(lib().spc3d_plan_create_csr(ctypes.byref(h), nnz, _ptr(rowptr), _ptr(col_gid),
                                       row_range[0], row_range[1], col_range[0], col_range[1],
                                       flags, _ptr(ws), ws.numel(), _stream(stream)),
           "spc3d_plan_create_csr")
    return Plan(h, ws, row_range, col_range, flags)


# ------------------------------------------------------------------ hot path

def gather(plan: Plan, axis: int, src: torch.Tensor, k0: int, kz: int,
           packed_dtype=torch.float32, out: torch.Tensor | None = None, stream=None):
    n = plan.R if axis == ROWS else plan.C
    rng = plan.row_range if axis == ROWS else plan.col_range
    if out is None:
        out = torch.empty((n, kz), dtype=packed_dtype, device=src.device)
    _need(src.dim() == 2 and src.stride(1) == 1, "src must be a row-major 2-D tensor")
    _need(src.shape[0] >= rng[1] - rng[0], "src needs one row per id of the axis range")
    _need(0 <= k0 and k0 + kz <= src.shape[1], "columns k0..k0+kz lie outside src")
    _need(out.is_contiguous() and out.numel() >= n * kz, "packed output too small")
    _check(lib().spc3d_gather(plan.handle, axis, _ptr(src), _dtype_code(src), src.stride(0), k0,
                              kz, _ptr(out), _dtype_code(out), _stream(stream)), "spc3d_gather")
    return out


def sddmm(plan: Plan, vals, A: torch.Tensor, B: torch.Tensor, kz: int | None = None,
          out: torch.Tensor | None = None, mode: int = OVERWRITE, variant: int = -1, stream=None):
    kz = A.shape[1] if kz is None else kz
    _need(A.dtype == B.dtype, "A and B must share a dtype")
    _need(A.is_contiguous() and B.is_contiguous(), "A and B must be packed (contiguous)")
    _need(A.numel() >= plan.R * kz and B.numel() >= plan.C * kz, "A or B too small for kz")
    _need(_rows_of(A, kz) and _rows_of(B, kz), "A and B must have kz columns")
    _need(vals is None or (vals.dtype == torch.float32 and vals.numel() >= plan.nnz),
          "vals must hold nnz FP32 values")
    if out is None:
        out = torch.empty(plan.nnz, dtype=torch.float32, device=A.device)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= plan.nnz,
          "out must hold nnz FP32 values")
    _check(lib().spc3d_sddmm(plan.handle, _ptr(vals), _ptr(A), _ptr(B), _dtype_code(A), kz,
                             _ptr(out), mode, variant, _stream(stream)), "spc3d_sddmm")
    return out


def spmm_buffer_size(plan: Plan, transpose: int, kz: int, variant: int = -1) -> int:
    b = ctypes.c_size_t()
    _check(lib().spc3d_spmm_buffer_size(plan.handle, transpose, kz, variant, ctypes.byref(b)),
           "spc3d_spmm_buffer_size")
    return b.value


def spmm(plan: Plan, vals, X: torch.Tensor, transpose: int = 0, kz: int | None = None,
         out: torch.Tensor | None = None, mode: int = OVERWRITE, variant: int = -1,
         buf: torch.Tensor | None = None, stream=None):
    kz = X.shape[1] if kz is None else kz
    n = plan.C if transpose else plan.R      # transpose 1 or 2: over columns
    nx = plan.R if transpose else plan.C
    _need(X.is_contiguous() and X.numel() >= nx * kz, "X too small for kz")
    _need(_rows_of(X, kz), "X must have kz columns")
    _need(vals is None or (vals.dtype == torch.float32 and vals.numel() >= plan.nnz),
          "vals must hold nnz FP32 values")
    if out is None:
        out = torch.empty((n, kz), dtype=torch.float32, device=X.device)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n * kz
          and _rows_of(out, kz), "out must hold n rows of kz FP32 values")
    need = spmm_buffer_size(plan, transpose, kz, variant)
    if buf is None:
        buf = plan.buffer(("spmm", transpose), need)
    _check(lib().spc3d_spmm(plan.handle, transpose, _ptr(vals), _ptr(X), _dtype_code(X), kz,
                            _ptr(out), mode, variant, _ptr(buf), buf.numel(), _stream(stream)),
           "spc3d_spmm")
    return out


def sddmm_spmm(plan: Plan, vals, A: torch.Tensor, B: torch.Tensor, kz: int | None = None,
               out: torch.Tensor | None = None, Y: torch.Tensor | None = None,
               mode: int = OVERWRITE, variant: int = -1, buf: torch.Tensor | None = None,
               stream=None):
    """SDDMM (slot-order out) and SpMM (Y = S B) in one pass; returns (out, Y)."""
    kz = A.shape[1] if kz is None else kz
    _need(A.dtype == B.dtype, "A and B must share a dtype")
    _need(A.is_contiguous() and B.is_contiguous(), "A and B must be packed (contiguous)")
    _need(A.numel() >= plan.R * kz and B.numel() >= plan.C * kz, "A or B too small for kz")
    _need(_rows_of(A, kz) and _rows_of(B, kz), "A and B must have kz columns")
    _need(vals is None or (vals.dtype == torch.float32 and vals.numel() >= plan.nnz),
          "vals must hold nnz FP32 values")
    if out is None:
        out = torch.empty(plan.nnz, dtype=torch.float32, device=A.device)
    if Y is None:
        Y = torch.empty((plan.R, kz), dtype=torch.float32, device=A.device)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= plan.nnz,
          "out must hold nnz FP32 values")
    _need(Y.dtype == torch.float32 and Y.is_contiguous() and Y.numel() >= plan.R * kz
          and _rows_of(Y, kz), "Y must hold R rows of kz FP32 values")
    need = spmm_buffer_size(plan, 0, kz, variant)
    if buf is None:
        buf = plan.buffer(("spmm", 0), need)
    _check(lib().spc3d_sddmm_spmm(plan.handle, _ptr(vals), _ptr(A), _ptr(B), _dtype_code(A), kz,
                                  _ptr(out), _ptr(Y), mode, variant, _ptr(buf), buf.numel(),
                                  _stream(stream)), "spc3d_sddmm_spmm")
    return out, Y


def sddmm_spmm_scatter(plan: Plan, vals, A: torch.Tensor, B: torch.Tensor, dst: torch.Tensor,
                       k0: int, kz: int | None = None, out: torch.Tensor | None = None,
                       out_mode: int = OVERWRITE, variant: int = -1,
                       buf: torch.Tensor | None = None, stream=None):
    """SDDMM into out (slot order) and the SpMM rows added into the owner's
    slab dst (rows gmap_r - row_lo, columns k0..k0+kz) in one pass: the fused
    pass and spc3d_scatter_reduce(ROWS) together.  Returns out."""
    kz = A.shape[1] if kz is None else kz
    _need(A.dtype == B.dtype, "A and B must share a dtype")
    _need(A.is_contiguous() and B.is_contiguous(), "A and B must be packed (contiguous)")
    _need(A.numel() >= plan.R * kz and B.numel() >= plan.C * kz, "A or B too small for kz")
    _need(_rows_of(A, kz) and _rows_of(B, kz), "A and B must have kz columns")
    _need(vals is None or (vals.dtype == torch.float32 and vals.numel() >= plan.nnz),
          "vals must hold nnz FP32 values")
    _need(dst.dim() == 2 and dst.stride(1) == 1 and dst.dtype == torch.float32,
          "dst must be a row-major FP32 2-D tensor")
    _need(dst.shape[0] >= plan.row_range[1] - plan.row_range[0],
          "dst needs one row per id of the row range")
    _need(0 <= k0 and k0 + kz <= dst.shape[1], "columns k0..k0+kz lie outside dst")
    if out is None:
        out = torch.empty(plan.nnz, dtype=torch.float32, device=A.device)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= plan.nnz,
          "out must hold nnz FP32 values")
    need = spmm_buffer_size(plan, 0, kz, variant)
    if buf is None:
        buf = plan.buffer(("spmm", 0), need)
    _check(lib().spc3d_sddmm_spmm_scatter(plan.handle, _ptr(vals), _ptr(A), _ptr(B),
                                          _dtype_code(A), kz, _ptr(out), out_mode, _ptr(dst),
                                          dst.stride(0), k0, variant, _ptr(buf), buf.numel(),
                                          _stream(stream)), "spc3d_sddmm_spmm_scatter")
    return out


def sddmm_spmm_static(plan: Plan, vals, A: torch.Tensor, B: torch.Tensor, kz: int | None = None,
                      out: torch.Tensor | None = None, Y: torch.Tensor | None = None,
                      mode: int = OVERWRITE, variant: int = -1, stream=None):
    """sddmm_spmm with the library's static scratch instead of a buffer argument
    (spc3d_sddmm_spmm_static); returns (out, Y).  The caller provides out and Y
    when nothing may be allocated."""
    kz = A.shape[1] if kz is None else kz
    _need(A.dtype == B.dtype, "A and B must share a dtype")
    _need(A.is_contiguous() and B.is_contiguous(), "A and B must be packed (contiguous)")
    _need(A.numel() >= plan.R * kz and B.numel() >= plan.C * kz, "A or B too small for kz")
    _need(_rows_of(A, kz) and _rows_of(B, kz), "A and B must have kz columns")
    _need(vals is None or (vals.dtype == torch.float32 and vals.numel() >= plan.nnz),
          "vals must hold nnz FP32 values")
    if out is None:
        out = torch.empty(plan.nnz, dtype=torch.float32, device=A.device)
    if Y is None:
        Y = torch.empty((plan.R, kz), dtype=torch.float32, device=A.device)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= plan.nnz,
          "out must hold nnz FP32 values")
    _need(Y.dtype == torch.float32 and Y.is_contiguous() and Y.numel() >= plan.R * kz
          and _rows_of(Y, kz), "Y must hold R rows of kz FP32 values")
    _check(lib().spc3d_sddmm_spmm_static(plan.handle, _ptr(vals), _ptr(A), _ptr(B),
                                         _dtype_code(A), kz, _ptr(out), _ptr(Y), mode, variant,
                                         _stream(stream)), "spc3d_sddmm_spmm_static")
    return out, Y


def scatter_reduce(plan: Plan, axis: int, packed: torch.Tensor, dst: torch.Tensor, k0: int,
                   stream=None):
    n = plan.R if axis == ROWS else plan.C
    rng = plan.row_range if axis == ROWS else plan.col_range
    _need(dst.dim() == 2 and dst.stride(1) == 1 and dst.dtype == torch.float32,
          "dst must be a row-major FP32 2-D tensor")
    _need(dst.shape[0] >= rng[1] - rng[0], "dst needs one row per id of the axis range")
    _need(packed.dtype == torch.float32 and packed.is_contiguous() and packed.dim() == 2
          and packed.shape[0] >= n, "packed must be [n, kz] FP32")
    _need(0 <= k0 and k0 + packed.shape[1] <= dst.shape[1], "columns k0..k0+kz lie outside dst")
    _check(lib().spc3d_scatter_reduce(plan.handle, axis, _ptr(packed), packed.shape[1],
                                      _ptr(dst), dst.stride(0), k0, _stream(stream)),
           "spc3d_scatter_reduce")
    return dst


def plan_check(plan: Plan, stream=None) -> None:
    """Checks the plan's local ids on the device (spc3d_plan_check); raises
    Spc3dError (ERR_OUT_OF_RANGE) naming the first violated invariant."""
    _check(lib().spc3d_plan_check(plan.handle, _stream(stream)), "spc3d_plan_check")


def debug_bounds() -> bool:
    """Whether SPC3D_DEBUG_BOUNDS makes every launching call check its plan."""
    return bool(lib().spc3d_debug_bounds())


def permute_values(plan: Plan, direction: int, x: torch.Tensor, out=None, stream=None):
    _need(x.dtype == torch.float32 and x.is_contiguous() and x.numel() >= plan.nnz,
          "x must hold nnz FP32 values")
    if out is None:
        out = torch.empty_like(x)
    _check(lib().spc3d_permute_values(plan.handle, direction, _ptr(x), _ptr(out),
                                      _stream(stream)), "spc3d_permute_values")
    return out


def row_softmax_buffer_size(plan: Plan) -> int:
    b = ctypes.c_size_t()
    _check(lib().spc3d_row_softmax_buffer_size(plan.handle, ctypes.byref(b)),
           "spc3d_row_softmax_buffer_size")
    return b.value


def row_softmax(plan: Plan, e: torch.Tensor, out=None, stream=None):
    _need(e.dtype == torch.float32 and e.is_contiguous() and e.numel() >= plan.nnz,
          "e must hold nnz FP32 values")
    out = torch.empty_like(e) if out is None else out
    buf = plan.buffer("softmax", row_softmax_buffer_size(plan))
    _check(lib().spc3d_row_softmax(plan.handle, _ptr(e), _ptr(out), _ptr(buf), buf.numel(),
                                   _stream(stream)), "spc3d_row_softmax")
    return out


def row_softmax_bwd(plan: Plan, alpha: torch.Tensor, dalpha: torch.Tensor, out=None, stream=None):
    _need(alpha.numel() >= plan.nnz and dalpha.numel() >= plan.nnz, "need nnz values")
    out = torch.empty_like(alpha) if out is None else out
    buf = plan.buffer("softmax", row_softmax_buffer_size(plan))
    _check(lib().spc3d_row_softmax_bwd(plan.handle, _ptr(alpha), _ptr(dalpha), _ptr(out),
                                       _ptr(buf), buf.numel(), _stream(stream)),
           "spc3d_row_softmax_bwd")
    return out


def row_softmax_apply(plan: Plan, e: torch.Tensor, stats: torch.Tensor, out=None, stream=None):
    """alpha[p] = exp(e[p] - stats[r, 0]) / stats[r, 1] for the entries p of row r."""
    _need(e.dtype == torch.float32 and e.is_contiguous() and e.numel() >= plan.nnz,
          "e must hold nnz FP32 values")
    _need(stats.dtype == torch.float32 and stats.is_contiguous() and stats.numel() >= 2 * plan.R,
          "stats must hold R (max, sum) FP32 pairs")
    out = torch.empty_like(e) if out is None else out
    _check(lib().spc3d_row_softmax_apply(plan.handle, _ptr(e), _ptr(stats), _ptr(out),
                                         _stream(stream)), "spc3d_row_softmax_apply")
    return out


def attention_fwd_buffer_size(plan: Plan, kz: int, dtype: int = F32, variant: int = -1) -> int:
    b = ctypes.c_size_t()
    _check(lib().spc3d_attention_fwd_buffer_size(plan.handle, kz, dtype, variant,
                                                 ctypes.byref(b)),
           "spc3d_attention_fwd_buffer_size")
    return b.value


def attention_supported(kz: int, dtype: int = F32, variant: int = -1) -> bool:
    """Whether spc3d_attention_fwd covers (kz, dtype, variant) (host-only check)."""
    nb = kz * (4 if dtype == F32 else 2)
    if variant >= 0:
        lanes = 1 << (variant & 15)
        nvec = nb // 16
        return nb % 16 == 0 and nvec % lanes == 0 and nvec // lanes in (1, 2)
    return nb in (64, 128, 256, 512)


def attention_fwd(plan: Plan, Q: torch.Tensor, K: torch.Tensor, V: torch.Tensor,
                  kz: int | None = None, out: torch.Tensor | None = None,
                  stats: torch.Tensor | None = None, want_stats: bool = True, variant: int = -1,
                  buf: torch.Tensor | None = None, stream=None):
    """Fused masked attention forward: out = rowsoftmax(SDDMM(Q, K)) . V in one pass.

    Returns (out [R, kz] FP32, stats [R, 2] FP32 (row max, row sum of exp) or None)."""
    kz = Q.shape[1] if kz is None else kz
    _need(Q.dtype == K.dtype == V.dtype, "Q, K and V must share a dtype")
    _need(Q.is_contiguous() and K.is_contiguous() and V.is_contiguous(),
          "Q, K and V must be packed (contiguous)")
    _need(Q.numel() >= plan.R * kz and K.numel() >= plan.C * kz and V.numel() >= plan.C * kz,
          "Q, K or V too small for kz")
    if out is None:
        out = torch.empty((plan.R, kz), dtype=torch.float32, device=Q.device)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= plan.R * kz,
          "out too small")
    if stats is None and want_stats:
        stats = torch.empty((plan.R, 2), dtype=torch.float32, device=Q.device)
    if stats is not None:
        _need(stats.dtype == torch.float32 and stats.is_contiguous()
              and stats.numel() >= 2 * plan.R, "stats must hold R (max, sum) pairs")
    dt = _dtype_code(Q)
    need = attention_fwd_buffer_size(plan, kz, dt, variant)
    if buf is None:
        buf = plan.buffer(("attention", kz), need)
    _check(lib().spc3d_attention_fwd(plan.handle, _ptr(Q), _ptr(K), _ptr(V), dt, kz, _ptr(out),
                                     _ptr(stats), variant, _ptr(buf), buf.numel(),
                                     _stream(stream)), "spc3d_attention_fwd")
    return out, stats


def lambda_owners(gmaps, lo: int, hi: int, rand: torch.Tensor | None = None,
                  device=None, stream=None) -> dict:
    """lambda counts and Algorithm 1 owners of ids [lo, hi) over the parts whose
    distinct ids are the int64 device tensors gmaps[p] (None or empty for a
    part that uses none).  rand: hi - lo uint64 draws (as int64) or None.
    Returns device tensors lambda_ (int32), owner (int32), owned (int64, one per
    part) and comm (int64 [nparts, nparts]: rows part p receives from part q)."""
    nparts = len(gmaps)
    _need(1 <= nparts <= 64, "1 to 64 parts")
    dev = device or next((g.device for g in gmaps if g is not None), torch.device("cuda"))
    for g in gmaps:
        if g is not None:
            _need(g.dtype == torch.int64 and g.is_contiguous(), "gmaps must be int64 contiguous")
    n = hi - lo
    if rand is not None:
        _need(rand.dtype in (torch.int64, torch.uint64) and rand.numel() >= n
              and rand.is_contiguous(), "rand must hold hi - lo 64-bit draws")
    ptrs = (ctypes.c_void_p * nparts)(*[None if g is None or g.numel() == 0 else g.data_ptr()
                                        for g in gmaps])
    counts = (ctypes.c_int64 * nparts)(*[0 if g is None else g.numel() for g in gmaps])
    lam = torch.empty(n, dtype=torch.int32, device=dev)
    owner = torch.empty(n, dtype=torch.int32, device=dev)
    owned = torch.empty(nparts, dtype=torch.int64, device=dev)
    comm = torch.empty((nparts, nparts), dtype=torch.int64, device=dev)
    b = ctypes.c_size_t()
    _check(lib().spc3d_lambda_owners_workspace_size(lo, hi, ctypes.byref(b)),
           "spc3d_lambda_owners_workspace_size")
    ws = torch.empty(b.value, dtype=torch.uint8, device=dev)
    _check(lib().spc3d_lambda_owners(nparts, ctypes.cast(ptrs, ctypes.c_void_p),
                                     ctypes.cast(counts, ctypes.c_void_p), lo, hi, _ptr(rand),
                                     _ptr(lam), _ptr(owner), _ptr(owned), _ptr(comm), _ptr(ws),
                                     ws.numel(), _stream(stream)), "spc3d_lambda_owners")
    return dict(lambda_=lam, owner=owner, owned=owned, comm=comm)


def mul_values(plan: Plan, a: torch.Tensor, b: torch.Tensor, out=None, stream=None):
    _need(a.numel() >= plan.nnz and b.numel() >= plan.nnz, "need nnz values")
    _need(a.dtype == torch.float32 and b.dtype == torch.float32, "FP32 values")
    out = torch.empty_like(a) if out is None else out
    _check(lib().spc3d_mul_values(plan.handle, _ptr(a), _ptr(b), _ptr(out), _stream(stream)),
           "spc3d_mul_values")
    return out


# ------------------------------------------------- learned variant selector

def variant_check(op: int, kz: int, dtype: int, variant: int) -> int:
    """Status of spc3d_variant_check (OK, ERR_UNSUPPORTED or ERR_INVALID_ARG); no launch."""
    return lib().spc3d_variant_check(op, kz, dtype, variant)


def plan_features(plan: Plan, kz: int, dtype: int, transpose: int = 0, out=None, stream=None):
    """SPC3D_NFEAT FP32 sparsity features of the plan (device tensor)."""
    dev = plan.ws.device
    if out is None:
        out = torch.empty(NFEAT, dtype=torch.float32, device=dev)
    _need(out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= NFEAT,
          "out must hold NFEAT FP32 values")
    buf = plan.buffer("features", FEATURES_BUFFER_BYTES)
    _check(lib().spc3d_plan_features(plan.handle, transpose, kz, dtype, _ptr(out), _ptr(buf),
                                     buf.numel(), _stream(stream)), "spc3d_plan_features")
    return out


def _f32_2d(t, rows, cols, name):
    _need(t.dtype == torch.float32 and t.is_contiguous() and t.numel() >= rows * cols,
          f"{name} must be a contiguous FP32 [{rows} x {cols}] tensor")


def mlp_linear_fwd(X: torch.Tensor, W: torch.Tensor, b=None, relu: bool = False, out=None,
                   stream=None):
    n, fin = X.shape
    fout = W.shape[0]
    _f32_2d(X, n, fin, "X")
    _f32_2d(W, fout, fin, "W")
    _need(W.shape[1] == fin, "W must be [fout x fin]")
    _need(b is None or (b.dtype == torch.float32 and b.numel() == fout), "b must hold fout values")
    if out is None:
        out = torch.empty((n, fout), dtype=torch.float32, device=X.device)
    _f32_2d(out, n, fout, "out")
    _check(lib().spc3d_mlp_linear_fwd(n, fin, fout, _ptr(X), _ptr(W), _ptr(b), _ptr(out),
                                      int(relu), _stream(stream)), "spc3d_mlp_linear_fwd")
    return out


def mlp_linear_bwd_buffer_size(n: int, fin: int, fout: int) -> int:
    b = ctypes.c_size_t()
    _check(lib().spc3d_mlp_linear_bwd_buffer_size(n, fin, fout, ctypes.byref(b)),
           "spc3d_mlp_linear_bwd_buffer_size")
    return b.value


def mlp_linear_bwd(X, W, Y, dY, relu: bool = False, need_dx: bool = True, dX=None, dW=None,
                   db=None, buf=None, stream=None):
    """Returns (dX or None, dW, db) of mlp_linear_fwd."""
    n, fin = X.shape
    fout = W.shape[0]
    _f32_2d(X, n, fin, "X")
    _f32_2d(W, fout, fin, "W")
    _f32_2d(dY, n, fout, "dY")
    _need(not relu or Y is not None, "Y is needed with relu")
    if relu:
        _f32_2d(Y, n, fout, "Y")
    dev = X.device
    if need_dx and dX is None:
        dX = torch.empty((n, fin), dtype=torch.float32, device=dev)
    if dW is None:
        dW = torch.empty((fout, fin), dtype=torch.float32, device=dev)
    if db is None:
        db = torch.empty(fout, dtype=torch.float32, device=dev)
    need = mlp_linear_bwd_buffer_size(n, fin, fout)
    if buf is None or buf.numel() < need:
        buf = torch.empty(need, dtype=torch.uint8, device=dev)
    _check(lib().spc3d_mlp_linear_bwd(n, fin, fout, _ptr(X), _ptr(W), _ptr(Y if relu else None),
                                      _ptr(dY), int(relu), _ptr(dX if need_dx else None),
                                      _ptr(dW), _ptr(db), _ptr(buf), buf.numel(),
                                      _stream(stream)), "spc3d_mlp_linear_bwd")
    return (dX if need_dx else None), dW, db


def mlp_mse(P, T, M, dP=None, loss=None, stream=None):
    """Masked mean squared error; returns (loss [1] device tensor, dP)."""
    n = P.numel()
    for t, name in ((P, "P"), (T, "T"), (M, "M")):
        _need(t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n,
              f"{name} must be contiguous FP32 with {n} values")
    dP = torch.empty_like(P) if dP is None else dP
    loss = torch.empty(1, dtype=torch.float32, device=P.device) if loss is None else loss
    _check(lib().spc3d_mlp_mse(n, _ptr(P), _ptr(T), _ptr(M), _ptr(dP), _ptr(loss),
                               _stream(stream)), "spc3d_mlp_mse")
    return loss, dP


def mlp_adam(w, g, m, v, lr: float, beta1: float, beta2: float, eps: float, step: int,
             stream=None):
    n = w.numel()
    for t, name in ((w, "w"), (g, "g"), (m, "m"), (v, "v")):
        _need(t.dtype == torch.float32 and t.is_contiguous() and t.numel() == n,
              f"{name} must be contiguous FP32 with {n} values")
    _check(lib().spc3d_mlp_adam(n, _ptr(w), _ptr(g), _ptr(m), _ptr(v), lr, beta1, beta2, eps,
                                step, _stream(stream)), "spc3d_mlp_adam")
    return w


def mlp_masked_argmin(P, M, pref: int = -1, margin: float = 0.0, out=None, stream=None):
    """Per row the least-P allowed column, or pref when it is allowed and within
    margin of that least value (spc3d_mlp_masked_argmin)."""
    n, m = P.shape
    _f32_2d(P, n, m, "P")
    _f32_2d(M, n, m, "M")
    out = torch.empty(n, dtype=torch.int32, device=P.device) if out is None else out
    _check(lib().spc3d_mlp_masked_argmin(n, m, _ptr(P), _ptr(M), pref, margin, _ptr(out),
                                         _stream(stream)),
           "spc3d_mlp_masked_argmin")
    return out
