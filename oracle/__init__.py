"""FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.  The C
part (``oracle.c``) is built with gcc, without fast-math and with FP
contraction off, into ``liboracle.so``; a few steps (the selector MLP) are
plain NumPy float64.  Nothing here is shared with the HIP library.

Every function cites the passage of the paper it follows (see oracle.c).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SO names another build of oracle.c (the tests' sanitizer build)
_SO = os.environ.get("ORACLE_SO") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
               "-fno-fast-math", os.path.join(_HERE, "oracle.c"), "-lm", "-o", _SO + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _p(a):
    return None if a is None else a.ctypes.data


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_relabel.restype = ctypes.c_int
        lib.oracle_relabel.argtypes = [i64, vp, vp, i64, i64, i64, i64, vp, vp, vp, vp, vp, vp,
                                       vp, vp, vp, vp, vp, vp]
        lib.oracle_relabel_grouped.restype = ctypes.c_int
        lib.oracle_relabel_grouped.argtypes = [i64, vp, vp, i64, i64, i64, i64, vp,
                                               ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp,
                                               vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.oracle_gather_f32.restype = None
        lib.oracle_gather_f32.argtypes = [i64, vp, i64, vp, i64, i64, i64, vp]
        lib.oracle_gather_bf16.restype = None
        lib.oracle_gather_bf16.argtypes = [i64, vp, i64, vp, i64, i64, i64, vp]
        lib.oracle_bf16_rne.restype = ctypes.c_uint16
        lib.oracle_bf16_rne.argtypes = [ctypes.c_float]
        lib.oracle_bf16_rne_array.restype = None
        lib.oracle_bf16_rne_array.argtypes = [i64, vp, vp]
        lib.oracle_scatter_add_f32.restype = None
        lib.oracle_scatter_add_f32.argtypes = [i64, vp, i64, vp, i64, vp, i64, i64]
        lib.oracle_sddmm.restype = None
        lib.oracle_sddmm.argtypes = [i64, vp, vp, i64, i64, vp, vp, i64, vp, i64, i64, i64, vp, vp]
        lib.oracle_spmm.restype = None
        lib.oracle_spmm.argtypes = [i64, vp, vp, i64, i64, vp, i64, vp, vp, i64, i64, i64, vp, vp]
        lib.oracle_attention_fwd.restype = None
        lib.oracle_attention_fwd.argtypes = [i64, vp, vp, i64, vp, vp, vp, vp, vp, vp]
        lib.oracle_attention_bwd.restype = None
        lib.oracle_attention_bwd.argtypes = [i64, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp,
                                             vp, vp]
        lib.oracle_lambda_owners.restype = None
        lib.oracle_lambda_owners.argtypes = [ctypes.c_int, vp, vp, i64, i64, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ------------------------------------------------------------------ relabel

def relabel(rows, cols, row_range, col_range, csc: bool = False, group_r=None, ngroups_r=0,
            group_c=None, ngroups_c=0) -> dict:
    """Localization of a block (paper: Section "Data distribution").

    Returns gmap_r, gmap_c (int64), lmap_r, lmap_c, rowptr, colidx, perm
    (int32) and, with csc=True, colptr, rowidx_t, slot_t.  With group_r
    (int32 key per id of the row range, keys in [0, ngroups_r)) local rows are
    ordered by (key, global id), the owner-grouped order of SpC-RB; likewise
    for columns.  Raises ValueError on an id outside its range or a key
    outside [0, ngroups).
    """
    lib = _load()
    gr = None if group_r is None else _c(group_r, np.int32)
    gc = None if group_c is None else _c(group_c, np.int32)
    rows = _c(rows, np.int64)
    cols = _c(cols, np.int64)
    nnz = rows.shape[0]
    rr = row_range[1] - row_range[0]
    cr = col_range[1] - col_range[0]
    gmap_r = np.empty(max(min(nnz, rr), 1), np.int64)
    gmap_c = np.empty(max(min(nnz, cr), 1), np.int64)
    lmap_r = np.empty(max(rr, 1), np.int32)
    lmap_c = np.empty(max(cr, 1), np.int32)
    rowptr = np.empty(max(min(nnz, rr), 0) + 1, np.int32)
    colidx = np.empty(max(nnz, 1), np.int32)
    perm = np.empty(max(nnz, 1), np.int32)
    colptr = rowidx_t = slot_t = None
    if csc:
        colptr = np.empty(max(min(nnz, cr), 0) + 1, np.int32)
        rowidx_t = np.empty(max(nnz, 1), np.int32)
        slot_t = np.empty(max(nnz, 1), np.int32)
    R = ctypes.c_int64()
    C = ctypes.c_int64()
    rc = lib.oracle_relabel_grouped(nnz, _p(rows), _p(cols), row_range[0], row_range[1],
                                    col_range[0], col_range[1], _p(gr), ngroups_r, _p(gc),
                                    ngroups_c, ctypes.byref(R), ctypes.byref(C), _p(gmap_r),
                                    _p(gmap_c), _p(lmap_r), _p(lmap_c), _p(rowptr), _p(colidx),
                                    _p(perm), _p(colptr), _p(rowidx_t), _p(slot_t))
    if rc == -2:
        raise ValueError("group key outside [0, ngroups)")
    if rc != 0:
        raise ValueError("global id outside its range")
    R, C = R.value, C.value
    out = dict(R=R, C=C, gmap_r=gmap_r[:R], gmap_c=gmap_c[:C], lmap_r=lmap_r[:rr],
               lmap_c=lmap_c[:cr], rowptr=rowptr[:R + 1], colidx=colidx[:nnz],
               perm=perm[:nnz])
    if csc:
        out.update(colptr=colptr[:C + 1], rowidx_t=rowidx_t[:nnz], slot_t=slot_t[:nnz])
    return out


# ------------------------------------------------------------ pack / unpack

def gather_f32(gmap, lo, src, k0, kz):
    """SpC-BB packing (paper: Section "Sparse communication model", Method 1)."""
    gmap = _c(gmap, np.int64)
    src = _c(src, np.float32)
    n = gmap.shape[0]
    out = np.empty((n, kz), np.float32)
    _load().oracle_gather_f32(n, _p(gmap), lo, _p(src), src.shape[1], k0, kz, _p(out))
    return out


def bf16_rne(x) -> np.ndarray:
    """FP32 -> bfloat16 bit patterns (uint16), nearest-even, from the format's definition."""
    x = _c(x, np.float32)
    out = np.empty(x.shape, np.uint16)
    _load().oracle_bf16_rne_array(x.size, _p(x), _p(out))
    return out


def bf16_to_f32(u16) -> np.ndarray:
    """Widen bfloat16 bit patterns to FP32 (exact)."""
    u16 = np.asarray(u16, dtype=np.uint16)
    return (u16.astype(np.uint32) << 16).view(np.float32)


def gather_bf16(gmap, lo, src, k0, kz):
    gmap = _c(gmap, np.int64)
    src = _c(src, np.float32)
    n = gmap.shape[0]
    out = np.empty((n, kz), np.uint16)
    _load().oracle_gather_bf16(n, _p(gmap), lo, _p(src), src.shape[1], k0, kz, _p(out))
    return out


def scatter_add_f32(gmap, lo, packed, dst, k0):
    """SpC-BB unpacking with reduction into dst (modified in place, FP32 adds)."""
    gmap = _c(gmap, np.int64)
    packed = _c(packed, np.float32)
    assert dst.dtype == np.float32 and dst.flags.c_contiguous
    n, kz = packed.shape if packed.ndim == 2 else (gmap.shape[0], 0)
    _load().oracle_scatter_add_f32(n, _p(gmap), lo, _p(packed), kz, _p(dst), dst.shape[1], k0)
    return dst


# ------------------------------------------------------------------ compute

def sddmm(rows, cols, row_lo, col_lo, vals, A, B, k0, kz):
    """Eq. (1) in caller order; returns (out, mag) as float64 arrays."""
    rows = _c(rows, np.int64)
    cols = _c(cols, np.int64)
    A = _c(A, np.float32)
    B = _c(B, np.float32)
    v = None if vals is None else _c(vals, np.float32)
    nnz = rows.shape[0]
    out = np.empty(max(nnz, 1), np.float64)
    mag = np.empty(max(nnz, 1), np.float64)
    _load().oracle_sddmm(nnz, _p(rows), _p(cols), row_lo, col_lo, _p(v), _p(A), A.shape[1],
                         _p(B), B.shape[1], k0, kz, _p(out), _p(mag))
    return out[:nnz], mag[:nnz]


def spmm(rows, cols, row_lo, col_lo, lmap_r, R, vals, B, k0, kz):
    """Eq. (2) over local rows; returns (Y, mag) as [R, kz] float64 arrays."""
    rows = _c(rows, np.int64)
    cols = _c(cols, np.int64)
    lmap_r = _c(lmap_r, np.int32)
    B = _c(B, np.float32)
    v = None if vals is None else _c(vals, np.float32)
    Y = np.empty((max(R, 1), kz), np.float64)
    mag = np.empty((max(R, 1), kz), np.float64)
    _load().oracle_spmm(rows.shape[0], _p(rows), _p(cols), row_lo, col_lo, _p(lmap_r), R,
                        _p(v), _p(B), B.shape[1], k0, kz, _p(Y), _p(mag))
    return Y[:R], mag[:R]


# ------------------------------------------------------------- attention

def attention_fwd(rowptr, colidx, Q, Kf, V):
    """Masked row-softmax attention; returns (e, alpha, out) in float64."""
    rowptr = _c(rowptr, np.int32)
    colidx = _c(colidx, np.int32)
    Q = _c(Q, np.float64)
    Kf = _c(Kf, np.float64)
    V = _c(V, np.float64)
    R, K = Q.shape
    nnz = colidx.shape[0]
    e = np.empty(max(nnz, 1))
    alpha = np.empty(max(nnz, 1))
    out = np.empty((max(R, 1), K))
    _load().oracle_attention_fwd(R, _p(rowptr), _p(colidx), K, _p(Q), _p(Kf), _p(V), _p(e),
                                 _p(alpha), _p(out))
    return e[:nnz], alpha[:nnz], out[:R]


def attention_bwd(rowptr, colidx, Q, Kf, V, alpha, dout):
    """Chain-rule gradients of attention_fwd; returns (de, dQ, dKf, dV)."""
    rowptr = _c(rowptr, np.int32)
    colidx = _c(colidx, np.int32)
    Q = _c(Q, np.float64)
    Kf = _c(Kf, np.float64)
    V = _c(V, np.float64)
    alpha = _c(alpha, np.float64)
    dout = _c(dout, np.float64)
    R, K = Q.shape
    C = Kf.shape[0]
    nnz = colidx.shape[0]
    de = np.empty(max(nnz, 1))
    dQ = np.empty((max(R, 1), K))
    dKf = np.empty((max(C, 1), K))
    dV = np.empty((max(C, 1), K))
    _load().oracle_attention_bwd(R, C, _p(rowptr), _p(colidx), K, _p(Q), _p(Kf), _p(V),
                                 _p(alpha), _p(dout), _p(de), _p(dQ), _p(dKf), _p(dV))
    return de[:nnz], dQ[:R], dKf[:C], dV[:C]


# ------------------------------------------- lambda and Algorithm 1 owners

def lambda_owners(gmaps, lo, hi, rnd=None) -> dict:
    """lambda, Algorithm 1 owners, owned counts and the receive matrix of one
    block row whose part p uses the distinct ids gmaps[p] (see the C source)."""
    nparts = len(gmaps)
    arrs = [_c(g, np.int64) for g in gmaps]
    counts = np.array([a.shape[0] for a in arrs], dtype=np.int64)
    ptrs = (ctypes.c_void_p * nparts)(*[a.ctypes.data for a in arrs])
    n = hi - lo
    lam = np.empty(max(n, 1), np.int32)
    owner = np.empty(max(n, 1), np.int32)
    owned = np.empty(nparts, np.int64)
    comm = np.empty(nparts * nparts, np.int64)
    r = None if rnd is None else _c(rnd, np.uint64)
    _load().oracle_lambda_owners(nparts, ctypes.cast(ptrs, ctypes.c_void_p), _p(counts), lo, hi,
                                 None if r is None else _p(r), _p(lam), _p(owner), _p(owned),
                                 _p(comm))
    return dict(lambda_=lam[:n], owner=owner[:n], owned=owned,
                comm=comm.reshape(nparts, nparts))
