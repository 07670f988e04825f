"""Seeded synthetic inputs (input tooling only; no method arithmetic).

The shared library ``libsynth.so`` is built from ``synth.c`` with gcc by
:func:`build`.  Everything returned here is a NumPy array on the host, so the
same inputs feed the CPU oracle and the GPU path.

Workload recipes
----------------
``tiny``      4096 x 4096, exactly 40,000 distinct uniform positions, values
              U[-1,1), A and B 4096 x 32, single block whose global ids equal
              its local ids.
``share3d``   R-MAT (a=0.57, b=c=0.19, d=0.05) on 2^24 vertices with 2^28
              edge samples (average degree 16), Graph500-style vertex
              permutation, de-duplicated; block (5,2) of the 8 x 8 grid, so
              row ids lie in [5*2^21, 6*2^21) and column ids in
              [2*2^21, 3*2^21).  Dense A and B slabs 2^21 x 128, local K-slice
              z=1 of 4 (k0=32, kz=32).
``share3d_uniform`` the same block shape, ranges, dense slabs and K-slice
              with 4,012,517 distinct uniform positions (flat degrees).
``precision`` R-MAT on 2^22 vertices, 2^27 samples (average degree 32), the
              whole matrix as one block, K=128.
``attention`` R-MAT on 2^20 vertices, 2^25 samples, K=64.
``selector``  512 square blocks n x n for training and judging the learned
              variant selector: n = round(2^(10 + 8u)) (log-uniform in
              [2^10, 2^18]), target average degree 4 * 16^v (log-uniform in
              [4, 64]), u and v counter draws; even blocks take uniform
              positions (round(deg * n) distinct entries), odd blocks R-MAT on
              2^ceil(log2 n) vertices, permuted, keeping the ids below n, with
              deg * n * (2^s / n)^2 samples so that about deg * n land in the
              block before de-duplication.  Split 384 / 128 by block.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SYNTH_SO names another build of synth.c (the tests' sanitizer build)
_SO = os.environ.get("SYNTH_SO") or os.path.join(_HERE, "libsynth.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile libsynth.so with gcc (OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
               os.path.join(_HERE, "synth.c"), "-o", _SO + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, u64, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        pp = ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))
        lib.synth_draw.restype = u64
        lib.synth_draw.argtypes = [u64, u64]
        lib.synth_uniform_f32.restype = None
        lib.synth_uniform_f32.argtypes = [u64, u64, i64, ctypes.c_void_p]
        lib.synth_dense_f32.restype = None
        lib.synth_dense_f32.argtypes = [u64, i64, i64, i64, i64, i64, ctypes.c_void_p]
        lib.synth_rmat_block.restype = i64
        lib.synth_rmat_block.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64, ctypes.c_int,
                                         i64, i64, i64, i64, pp, pp]
        lib.synth_uniform_block.restype = i64
        lib.synth_uniform_block.argtypes = [i64, i64, i64, u64, i64, i64, pp, pp]
        lib.synth_draws_u64.restype = None
        lib.synth_draws_u64.argtypes = [u64, u64, i64, ctypes.c_void_p]
        lib.synth_free.restype = None
        lib.synth_free.argtypes = [ctypes.c_void_p]
        lib.synth_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def draw(seed: int, ctr: int) -> int:
    return int(_load().synth_draw(seed, ctr))


def draws_u64(seed: int, n: int, ctr0: int = 0) -> np.ndarray:
    """n raw 64-bit counter draws (seed, ctr0 + i)."""
    out = np.empty(n, dtype=np.uint64)
    _load().synth_draws_u64(seed, ctr0, n, out.ctypes.data)
    return out


def uniform_f32(seed: int, n: int, ctr0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _load().synth_uniform_f32(seed, ctr0, n, out.ctypes.data)
    return out


def dense_f32(seed: int, row0: int, nrows: int, ncols: int, gcols: int | None = None) -> np.ndarray:
    """Rows [row0, row0+nrows) of the seeded U[-1,1) matrix with gcols columns
    (first ``ncols`` columns materialised)."""
    gcols = ncols if gcols is None else gcols
    out = np.empty((nrows, ncols), dtype=np.float32)
    _load().synth_dense_f32(seed, row0, nrows, ncols, gcols, ncols, out.ctypes.data)
    return out


def _take(n, rp, cp):
    lib = _load()
    rows = np.ctypeslib.as_array(rp, shape=(max(n, 1),))[:n].copy()
    cols = np.ctypeslib.as_array(cp, shape=(max(n, 1),))[:n].copy()
    lib.synth_free(ctypes.cast(rp, ctypes.c_void_p))
    lib.synth_free(ctypes.cast(cp, ctypes.c_void_p))
    return rows, cols


def rmat_block(scale: int, nsamples: int, seed: int, row_range, col_range,
               abc=RMAT_ABC, permute: bool = True):
    """Distinct R-MAT entries inside one block, global ids, caller order."""
    lib = _load()
    rp = ctypes.POINTER(ctypes.c_int64)()
    cp = ctypes.POINTER(ctypes.c_int64)()
    n = lib.synth_rmat_block(scale, nsamples, abc[0], abc[1], abc[2], seed, int(permute),
                             row_range[0], row_range[1], col_range[0], col_range[1],
                             ctypes.byref(rp), ctypes.byref(cp))
    return _take(n, rp, cp)


def uniform_block(nrows: int, ncols: int, nnz: int, seed: int, row_lo: int = 0, col_lo: int = 0):
    """Exactly nnz distinct uniform positions (rejection), caller = draw order."""
    lib = _load()
    rp = ctypes.POINTER(ctypes.c_int64)()
    cp = ctypes.POINTER(ctypes.c_int64)()
    n = lib.synth_uniform_block(nrows, ncols, nnz, seed, row_lo, col_lo,
                                ctypes.byref(rp), ctypes.byref(cp))
    if n < 0:
        raise ValueError("nnz exceeds the number of cells")
    return _take(n, rp, cp)


def banded_block(lo: int, n: int, per_row: int, half_width: int, seed: int):
    """Distinct entries of a banded block over ids [lo, lo + n) on both axes:
    row i draws per_row columns i + U{-half_width, ..., half_width} (clipped
    to the range), duplicates dropped, caller order = draw order.  Counter
    draws (seed, i * per_row + t); the offset is the multiply-shift of the
    draw's high 32 bits onto 2 * half_width + 1 values."""
    d = draws_u64(seed, n * per_row)
    span = np.uint64(2 * half_width + 1)
    off = (((d >> np.uint64(32)) * span) >> np.uint64(32)).astype(np.int64) - half_width
    rows = np.repeat(np.arange(n, dtype=np.int64), per_row)
    cols = np.clip(rows + off, 0, n - 1)
    _, first = np.unique(rows * n + cols, return_index=True)
    keep = np.sort(first)
    return rows[keep] + lo, cols[keep] + lo


@dataclass
class Problem:
    """One local block plus the dense slabs it reads and writes.

    rows/cols: int64 global ids in caller order; vals: float32 caller order;
    A_src: [row_hi-row_lo, K] rows of A for the block's row range;
    B_src: [col_hi-col_lo, K] rows of B for the column range;
    k0, kz: the local K-slice.
    """
    name: str
    rows: np.ndarray
    cols: np.ndarray
    vals: np.ndarray
    row_range: tuple
    col_range: tuple
    A_src: np.ndarray
    B_src: np.ndarray
    K: int
    k0: int
    kz: int
    seed: int

    @property
    def nnz(self) -> int:
        return int(self.rows.shape[0])


def _dense_pair(seed, row_range, col_range, K):
    A = dense_f32(seed + 101, row_range[0], row_range[1] - row_range[0], K)
    B = dense_f32(seed + 202, col_range[0], col_range[1] - col_range[0], K)
    return A, B


def tiny(seed: int = 2404) -> Problem:
    n, nnz, K = 4096, 40_000, 32
    rows, cols = uniform_block(n, n, nnz, seed)
    vals = uniform_f32(seed + 7, rows.shape[0])
    A, B = _dense_pair(seed, (0, n), (0, n), K)
    return Problem("tiny", rows, cols, vals, (0, n), (0, n), A, B, K, 0, K, seed)


def share3d(seed: int = 2405, bx: int = 5, by: int = 2, z: int = 1, dense: bool = True) -> Problem:
    scale, deg, grid, Z, K = 24, 16, 8, 4, 128
    span = (1 << scale) // grid
    rr = (bx * span, (bx + 1) * span)
    cr = (by * span, (by + 1) * span)
    rows, cols = rmat_block(scale, deg << scale, seed, rr, cr)
    vals = uniform_f32(seed + 7, rows.shape[0])
    kz = K // Z
    if dense:
        A, B = _dense_pair(seed, rr, cr, K)
    else:
        A = B = None
    return Problem("share3d", rows, cols, vals, rr, cr, A, B, K, z * kz, kz, seed)


def share3d_uniform(seed: int = 2410, nnz: int = 4_012_517, bx: int = 5, by: int = 2,
                    z: int = 1, dense: bool = True) -> Problem:
    """The 3D-share block's shape (2^21 x 2^21 block (bx, by) of the 8 x 8 grid of
    2^24 ids, K = 128, K-slice z of 4) with nnz distinct uniform positions."""
    scale, grid, Z, K = 24, 8, 4, 128
    span = (1 << scale) // grid
    rr = (bx * span, (bx + 1) * span)
    cr = (by * span, (by + 1) * span)
    rows, cols = uniform_block(span, span, nnz, seed, rr[0], cr[0])
    vals = uniform_f32(seed + 7, rows.shape[0])
    kz = K // Z
    if dense:
        A, B = _dense_pair(seed, rr, cr, K)
    else:
        A = B = None
    return Problem("share3d_uniform", rows, cols, vals, rr, cr, A, B, K, z * kz, kz, seed)


def share3d_banded(seed: int = 2411, bxy: int = 2, per_row: int = 2, half_width: int = 1 << 14,
                   z: int = 1, dense: bool = True) -> Problem:
    """A diagonal block (bxy, bxy) of the 8 x 8 grid over 2^24 ids with a banded
    pattern (rows reuse nearby columns, as road and mesh graphs in their
    natural order do); slabs, K = 128 and the K-slice as for share3d."""
    scale, grid, Z, K = 24, 8, 4, 128
    span = (1 << scale) // grid
    rr = (bxy * span, (bxy + 1) * span)
    rows, cols = banded_block(rr[0], span, per_row, half_width, seed)
    vals = uniform_f32(seed + 7, rows.shape[0])
    kz = K // Z
    if dense:
        A, B = _dense_pair(seed, rr, rr, K)
    else:
        A = B = None
    return Problem("share3d_banded", rows, cols, vals, rr, rr, A, B, K, z * kz, kz, seed)


def rmat_whole(scale: int, deg: int, K: int, seed: int, name: str, dense: bool = True) -> Problem:
    n = 1 << scale
    rows, cols = rmat_block(scale, deg << scale, seed, (0, n), (0, n))
    vals = uniform_f32(seed + 7, rows.shape[0])
    if dense:
        A, B = _dense_pair(seed, (0, n), (0, n), K)
    else:
        A = B = None
    return Problem(name, rows, cols, vals, (0, n), (0, n), A, B, K, 0, K, seed)


def precision(seed: int = 2406, dense: bool = True) -> Problem:
    return rmat_whole(22, 32, 128, seed, "precision", dense)


def attention(seed: int = 2407, dense: bool = True) -> Problem:
    return rmat_whole(20, 32, 64, seed, "attention", dense)


def small_rmat(scale: int, deg: int, K: int, seed: int, row_range=None, col_range=None) -> Problem:
    """A small R-MAT block for tests (ragged tails, skewed rows)."""
    n = 1 << scale
    rr = row_range or (0, n)
    cr = col_range or (0, n)
    rows, cols = rmat_block(scale, deg << scale, seed, rr, cr)
    vals = uniform_f32(seed + 7, rows.shape[0])
    A, B = _dense_pair(seed, rr, cr, K)
    return Problem("small_rmat", rows, cols, vals, rr, cr, A, B, K, 0, K, seed)


SELECTOR_SEED = 2408


def _unit(seed: int, ctr: int) -> float:
    """Counter draw mapped to [0, 1) with 53 bits."""
    return (draw(seed, ctr) >> 11) * (1.0 / (1 << 53))


def selector_block(i: int, seed: int = SELECTOR_SEED, lg_lo: float = 10.0, lg_hi: float = 18.0,
                   deg_lo: float = 4.0, deg_hi: float = 64.0) -> dict:
    """Block i of the selector workload (see the module docstring).

    Returns dict(i, kind, n, deg, rows, cols): int64 ids in [0, n), caller order.
    """
    u = _unit(seed, 4 * i)
    v = _unit(seed, 4 * i + 1)
    n = int(round(2.0 ** (lg_lo + (lg_hi - lg_lo) * u)))
    deg = deg_lo * (deg_hi / deg_lo) ** v
    bseed = draw(seed, 4 * i + 2) & ((1 << 62) - 1)
    if i % 2 == 0:
        kind = "uniform"
        nnz = min(int(round(deg * n)), n * n // 2)
        rows, cols = uniform_block(n, n, nnz, bseed)
    else:
        kind = "rmat"
        s = max(1, (n - 1).bit_length())
        samples = int(round(deg * n * ((1 << s) / n) ** 2))
        rows, cols = rmat_block(s, samples, bseed, (0, n), (0, n))
    return dict(i=i, kind=kind, n=n, deg=deg, rows=rows, cols=cols)


def selector_split(nblocks: int = 512, ntrain: int = 384, seed: int = SELECTOR_SEED):
    """Seeded split of block indices into (train, held_out), both ascending."""
    order = sorted(range(nblocks), key=lambda i: (draw(seed + 1, i), i))
    return sorted(order[:ntrain]), sorted(order[ntrain:])
