"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something other than itself: a worked
example derived by hand, brute force on tiny inputs, dense library products
(NumPy float64), PyTorch's CPU bfloat16 rounding, closed forms and identities.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hand():
    with open(os.path.join(GOLDEN, "hand_example.json")) as f:
        return json.load(f)


# ----------------------------------------------------------------- relabel

def test_relabel_hand_example():
    g = _hand()
    out = oracle.relabel(g["rows"], g["cols"], g["row_range"], g["col_range"], csc=True)
    for key in ("gmap_r", "gmap_c", "lmap_r", "lmap_c", "rowptr", "colidx", "perm", "colptr",
                "rowidx_t", "slot_t"):
        np.testing.assert_array_equal(out[key], np.array(g[key]), err_msg=key)


def _brute_relabel(rows, cols, rr, cr):
    """Dictionary / sorted-list brute force of the localization rules."""
    gr = sorted(set(int(x) for x in rows))
    gc = sorted(set(int(x) for x in cols))
    lr_of = {g: i for i, g in enumerate(gr)}
    lc_of = {g: i for i, g in enumerate(gc)}
    lmap_r = [lr_of.get(g, -1) for g in range(rr[0], rr[1])]
    lmap_c = [lc_of.get(g, -1) for g in range(cr[0], cr[1])]
    ent = sorted((lr_of[int(r)], lc_of[int(c)], p) for p, (r, c) in enumerate(zip(rows, cols)))
    rowptr = [0] * (len(gr) + 1)
    for (r, _, _) in ent:
        rowptr[r + 1] += 1
    for i in range(len(gr)):
        rowptr[i + 1] += rowptr[i]
    slot_of = {p: q for q, (_, _, p) in enumerate(ent)}
    entT = sorted((lc_of[int(c)], lr_of[int(r)], p) for p, (r, c) in enumerate(zip(rows, cols)))
    colptr = [0] * (len(gc) + 1)
    for (c, _, _) in entT:
        colptr[c + 1] += 1
    for i in range(len(gc)):
        colptr[i + 1] += colptr[i]
    return dict(gmap_r=gr, gmap_c=gc, lmap_r=lmap_r, lmap_c=lmap_c, rowptr=rowptr,
                colidx=[c for (_, c, _) in ent], perm=[p for (_, _, p) in ent], colptr=colptr,
                rowidx_t=[r for (_, r, _) in entT], slot_t=[slot_of[p] for (_, _, p) in entT])


@pytest.mark.parametrize("seed,nnz,rr,cr,dup", [
    (1, 1, (0, 1), (0, 1), False),
    (2, 37, (100, 140), (7, 30), False),
    (3, 300, (0, 64), (0, 64), True),      # repeated (i,j) entries are separate tasks
    (4, 500, (5, 1005), (3000, 3013), True),
])
def test_relabel_brute_force(seed, nnz, rr, cr, dup):
    rng = np.random.default_rng(seed)
    rows = rng.integers(rr[0], rr[1], nnz)
    cols = rng.integers(cr[0], cr[1], nnz)
    if dup:
        rows[nnz // 2:] = rows[: nnz - nnz // 2]
        cols[nnz // 2:] = cols[: nnz - nnz // 2]
    out = oracle.relabel(rows, cols, rr, cr, csc=True)
    ref = _brute_relabel(rows, cols, rr, cr)
    for key, val in ref.items():
        np.testing.assert_array_equal(out[key], np.array(val, dtype=out[key].dtype), err_msg=key)


def test_relabel_empty_and_range_errors():
    out = oracle.relabel(np.zeros(0, np.int64), np.zeros(0, np.int64), (0, 8), (0, 4), csc=True)
    assert out["R"] == 0 and out["C"] == 0
    np.testing.assert_array_equal(out["rowptr"], [0])
    assert (out["lmap_r"] == -1).all() and (out["lmap_c"] == -1).all()
    with pytest.raises(ValueError):
        oracle.relabel([3, 8], [0, 1], (0, 8), (0, 4))
    with pytest.raises(ValueError):
        oracle.relabel([3], [-1], (0, 8), (0, 4))


def test_relabel_invariants_rmat_block():
    p = synth.small_rmat(14, 8, 8, 11, row_range=(1 << 13, 1 << 14), col_range=(0, 1 << 13))
    out = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range, csc=True)
    R, C = out["R"], out["C"]
    assert R == np.unique(p.rows).size and C == np.unique(p.cols).size
    assert (np.diff(out["gmap_r"]) > 0).all() and (np.diff(out["gmap_c"]) > 0).all()
    np.testing.assert_array_equal(out["lmap_r"][out["gmap_r"] - p.row_range[0]], np.arange(R))
    assert (out["lmap_r"] >= 0).sum() == R
    assert np.array_equal(np.sort(out["perm"]), np.arange(p.nnz))
    assert np.array_equal(np.sort(out["slot_t"]), np.arange(p.nnz))
    assert (np.diff(out["rowptr"]) >= 1).all() and out["rowptr"][-1] == p.nnz
    lr = np.repeat(np.arange(R), np.diff(out["rowptr"]))
    np.testing.assert_array_equal(out["gmap_r"][lr], p.rows[out["perm"]])
    np.testing.assert_array_equal(out["gmap_c"][out["colidx"]], p.cols[out["perm"]])
    # the column-major view names the same entries
    lc = np.repeat(np.arange(C), np.diff(out["colptr"]))
    np.testing.assert_array_equal(out["colidx"][out["slot_t"]], lc)
    np.testing.assert_array_equal(lr[out["slot_t"]], out["rowidx_t"])


# ----------------------------------------------------------- pack / unpack

def test_gather_scatter_hand_example():
    g = _hand()
    A = np.array(g["A_src"], np.float32)
    B = np.array(g["B_src"], np.float32)
    al = oracle.gather_f32(g["gmap_r"], g["row_range"][0], A, g["k0"], g["kz"])
    bl = oracle.gather_f32(g["gmap_c"], g["col_range"][0], B, g["k0"], g["kz"])
    np.testing.assert_array_equal(al, np.array(g["A_loc"], np.float32))
    np.testing.assert_array_equal(bl, np.array(g["B_loc"], np.float32))
    dst = np.zeros_like(A)
    oracle.scatter_add_f32(g["gmap_r"], g["row_range"][0], np.array(g["spmm_local_rows"],
                           np.float32), dst, g["k0"])
    want = np.zeros_like(A)
    want[[1, 3, 5], 1:3] = np.array(g["spmm_local_rows"], np.float32)
    np.testing.assert_array_equal(dst, want)


def test_scatter_of_gather_roundtrip_and_fp32_add():
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 24)).astype(np.float32)
    gmap = np.sort(rng.choice(300, 77, replace=False)).astype(np.int64) + 1000
    packed = oracle.gather_f32(gmap, 1000, X, 5, 11)
    dst = np.zeros_like(X)
    oracle.scatter_add_f32(gmap, 1000, packed, dst, 5)
    want = np.zeros_like(X)
    want[gmap - 1000, 5:16] = X[gmap - 1000, 5:16]
    np.testing.assert_array_equal(dst, want)
    # reduction is one IEEE binary32 add per element (NumPy float32 add is IEEE)
    base = rng.standard_normal((300, 24)).astype(np.float32)
    d2 = base.copy()
    oracle.scatter_add_f32(gmap, 1000, packed, d2, 5)
    want = base.copy()
    want[gmap - 1000, 5:16] = np.add(base[gmap - 1000, 5:16], packed, dtype=np.float32)
    np.testing.assert_array_equal(d2.view(np.uint32), want.view(np.uint32))


# ---------------------------------------------------------------- bfloat16

BF16_CASES = [  # (fp32 pattern, bf16 pattern), worked from the format definition
    (0x3F800000, 0x3F80),   # 1.0
    (0x3F808000, 0x3F80),   # 1 + 2^-8: tie, even neighbour is 0x3F80
    (0x3F818000, 0x3F82),   # 1 + 3*2^-8: tie, even neighbour is 0x3F82
    (0x3F808001, 0x3F81),   # just above the tie
    (0xBF808001, 0xBF81),   # sign symmetric
    (0x7F7FFFFF, 0x7F80),   # FLT_MAX rounds up to infinity
    (0x7F7F7FFF, 0x7F7F),   # below the tie at the top
    (0x7F7F8000, 0x7F80),   # tie with odd 0x7F7F rounds to infinity
    (0x00000001, 0x0000),   # smallest subnormal rounds to +0
    (0x00008000, 0x0000),   # tie between 0 and the smallest bf16 subnormal: even is 0
    (0x00018000, 0x0002),   # tie between 1 and 2 ulps: even is 2
    (0x00008001, 0x0001),
    (0x007FFFFF, 0x0080),   # largest fp32 subnormal rounds to the smallest normal
    (0x80000000, 0x8000),   # -0
    (0x7F800000, 0x7F80),   # +inf
    (0xFF800000, 0xFF80),   # -inf
    (0x7FC00000, 0x7FC0),   # quiet NaN
    (0x7F800001, 0x7FC0),   # signalling NaN becomes quiet
    (0xFF800001, 0xFFC0),   # sign kept
]


@pytest.mark.parametrize("pat,want", BF16_CASES)
def test_bf16_hand_cases(pat, want):
    x = np.array([pat], np.uint32).view(np.float32)
    assert int(oracle.bf16_rne(x)[0]) == want


def test_bf16_matches_torch_cpu_rounding():
    import torch
    rng = np.random.default_rng(7)
    pats = np.concatenate([
        rng.integers(0, 1 << 32, 1 << 22, dtype=np.uint64).astype(np.uint32),
        np.arange(0, 1 << 32, 4099, dtype=np.uint64).astype(np.uint32),
        # every low-half pattern around ties, for a spread of exponents
        (np.arange(0, 256, dtype=np.uint32)[:, None] << 23 |
         np.array([0x7FFF, 0x8000, 0x8001, 0x18000, 0x17FFF, 0xFFFF], np.uint32)[None, :]).ravel(),
    ])
    x = pats.view(np.float32)
    got = oracle.bf16_rne(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    np.testing.assert_array_equal(got[~nan], ref[~nan])
    assert np.isnan(oracle.bf16_to_f32(got[nan])).all()


def _bf16_chunk_vs_torch(lo, step):
    import torch
    pats = np.arange(lo, lo + step, dtype=np.int64).astype(np.uint32)
    x = pats.view(np.float32)
    got = oracle.bf16_rne(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    np.testing.assert_array_equal(got[~nan], ref[~nan], err_msg=f"chunk {lo:#x}")
    g = got[nan]
    assert ((g & 0x7F80) == 0x7F80).all() and ((g & 0x7F) != 0).all()
    assert np.array_equal(g >> 15, (pats[nan] >> 31).astype(np.uint16))


def test_bf16_all_fp32_patterns_against_torch_cpu():
    """Every one of the 2^32 FP32 bit patterns: the oracle's rounding equals
    PyTorch's CPU round-to-nearest-even conversion for all non-NaN inputs;
    NaNs stay NaNs with their sign.  Chunks run on threads (the oracle's C
    loop releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    step = 1 << 25
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_bf16_chunk_vs_torch, lo, step) for lo in range(0, 1 << 32, step)]:
            f.result()


# ------------------------------------------------------------------- SDDMM

def test_sddmm_spmm_hand_example():
    g = _hand()
    A = np.array(g["A_src"], np.float32)
    B = np.array(g["B_src"], np.float32)
    out, mag = oracle.sddmm(g["rows"], g["cols"], 10, 20, np.array(g["vals"], np.float32), A, B,
                            g["k0"], g["kz"])
    np.testing.assert_array_equal(out, g["sddmm_caller_order"])
    lm = oracle.relabel(g["rows"], g["cols"], g["row_range"], g["col_range"])
    Y, _ = oracle.spmm(g["rows"], g["cols"], 10, 20, lm["lmap_r"], lm["R"],
                       np.array(g["vals"], np.float32), B, g["k0"], g["kz"])
    np.testing.assert_array_equal(Y, g["spmm_local_rows"])
    assert out.sum() == g["sum_identity"]


def test_magnitude_sums_hand_example():
    """The magnitude sums M that every floating-point bar scales with: the
    hand-worked values (entry p1 of the SDDMM and row 15 of the SpMM cancel,
    so a magnitude taken as |value| fails here)."""
    g = _hand()
    A = np.array(g["A_src"], np.float32)
    B = np.array(g["B_src"], np.float32)
    vals = np.array(g["vals"], np.float32)
    _, mag = oracle.sddmm(g["rows"], g["cols"], 10, 20, vals, A, B, g["k0"], g["kz"])
    np.testing.assert_array_equal(mag, g["sddmm_mag"])
    lm = oracle.relabel(g["rows"], g["cols"], g["row_range"], g["col_range"])
    _, ymag = oracle.spmm(g["rows"], g["cols"], 10, 20, lm["lmap_r"], lm["R"], vals, B, g["k0"],
                          g["kz"])
    np.testing.assert_array_equal(ymag, g["spmm_mag"])


def _tiny_problem(seed, M=37, N=29, K=6, nnz=200, lo=(3, 50)):
    rng = np.random.default_rng(seed)
    flat = rng.choice(M * N, nnz, replace=False)
    rows = flat // N + lo[0]
    cols = flat % N + lo[1]
    vals = rng.uniform(-1, 1, nnz).astype(np.float32)
    A = rng.uniform(-1, 1, (M, K)).astype(np.float32)
    B = rng.uniform(-1, 1, (N, K)).astype(np.float32)
    return rows, cols, vals, A, B, (lo[0], lo[0] + M), (lo[1], lo[1] + N)


def test_sddmm_dense_masked_brute_force():
    rows, cols, vals, A, B, rr, cr = _tiny_problem(1)
    out, mag = oracle.sddmm(rows, cols, rr[0], cr[0], vals, A, B, 1, 4)
    dense = A[:, 1:5].astype(np.float64) @ B[:, 1:5].astype(np.float64).T   # library GEMM
    want = vals.astype(np.float64) * dense[rows - rr[0], cols - cr[0]]
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-15)
    assert (mag >= np.abs(out) - 1e-15).all()
    # M_p = |s_p| * sum_k |a_k b_k| over the slice only: the dense product of
    # the absolute values, sampled by the mask (each FP32 product is exact in
    # FP64, so only the order of four additions differs)
    absdense = (np.abs(A[:, 1:5].astype(np.float64)) @ np.abs(B[:, 1:5].astype(np.float64)).T)
    want_mag = np.abs(vals.astype(np.float64)) * absdense[rows - rr[0], cols - cr[0]]
    np.testing.assert_allclose(mag, want_mag, rtol=1e-15, atol=0)
    # the pin is sharp: with these signs |dot| < sum |a b| for most entries,
    # and the full-K sum differs from the slice's
    assert (np.abs(out) < mag * (1 - 1e-6)).mean() > 0.5
    full = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)).T
    assert not np.allclose(mag, np.abs(vals) * full[rows - rr[0], cols - cr[0]])


def test_sddmm_identity_pattern_is_diagonal():
    rng = np.random.default_rng(2)
    n, K = 50, 9
    A = rng.uniform(-1, 1, (n, K)).astype(np.float32)
    B = rng.uniform(-1, 1, (n, K)).astype(np.float32)
    idx = np.arange(n)
    out, _ = oracle.sddmm(idx, idx, 0, 0, None, A, B, 0, K)
    want = np.einsum("ik,ik->i", A.astype(np.float64), B.astype(np.float64))
    np.testing.assert_allclose(out, want, rtol=1e-15, atol=1e-15)


def test_sddmm_transpose_symmetry_and_kslices():
    rows, cols, vals, A, B, rr, cr = _tiny_problem(3, K=12)
    out, _ = oracle.sddmm(rows, cols, rr[0], cr[0], vals, A, B, 0, 12)
    outT, _ = oracle.sddmm(cols, rows, cr[0], rr[0], vals, B, A, 0, 12)
    np.testing.assert_allclose(outT, out, rtol=1e-14, atol=1e-15)
    # 3D split: Z instances over K/Z columns sum to the full-K result
    parts = [oracle.sddmm(rows, cols, rr[0], cr[0], vals, A, B, z * 3, 3)[0] for z in range(4)]
    np.testing.assert_allclose(sum(parts), out, rtol=1e-13, atol=1e-15)


# -------------------------------------------------------------------- SpMM

def test_spmm_dense_brute_force():
    rows, cols, vals, A, B, rr, cr = _tiny_problem(4)
    lm = oracle.relabel(rows, cols, rr, cr)
    Y, mag = oracle.spmm(rows, cols, rr[0], cr[0], lm["lmap_r"], lm["R"], vals, B, 2, 3)
    S = np.zeros((rr[1] - rr[0], cr[1] - cr[0]))
    S[rows - rr[0], cols - cr[0]] = vals
    dense = S @ B[:, 2:5].astype(np.float64)                               # library GEMM
    np.testing.assert_allclose(Y, dense[lm["gmap_r"] - rr[0]], rtol=0, atol=1e-14)
    assert (mag + 1e-15 >= np.abs(Y)).all()
    # M[l][k] = sum_p |s_p b_k|: |S| |B| over the slice, at the local rows
    absdense = np.abs(S) @ np.abs(B[:, 2:5].astype(np.float64))
    np.testing.assert_allclose(mag, absdense[lm["gmap_r"] - rr[0]], rtol=1e-14, atol=0)
    assert (np.abs(Y) < mag * (1 - 1e-6)).mean() > 0.5


def test_spmm_permutation_pattern_returns_rows_exactly():
    rng = np.random.default_rng(6)
    n, K = 64, 7
    B = rng.standard_normal((n, K)).astype(np.float32)
    sigma = rng.permutation(n)
    rows = np.arange(n)
    lm = oracle.relabel(rows, sigma, (0, n), (0, n))
    Y, _ = oracle.spmm(rows, sigma, 0, 0, lm["lmap_r"], lm["R"], None, B, 0, K)
    np.testing.assert_array_equal(Y, B[sigma].astype(np.float64))


def test_sum_identity_and_adjoint():
    """sum(SDDMM(S,A,B)) = trace(A^T SpMM(S,B)) and <X, S B> = <S^T X, B>."""
    rows, cols, vals, A, B, rr, cr = _tiny_problem(8, K=5)
    lm = oracle.relabel(rows, cols, rr, cr)
    out, mag = oracle.sddmm(rows, cols, rr[0], cr[0], vals, A, B, 0, 5)
    Y, _ = oracle.spmm(rows, cols, rr[0], cr[0], lm["lmap_r"], lm["R"], vals, B, 0, 5)
    Aloc = A[lm["gmap_r"] - rr[0]].astype(np.float64)
    np.testing.assert_allclose(out.sum(), (Aloc * Y).sum(), rtol=1e-13, atol=1e-13)
    lmT = oracle.relabel(cols, rows, cr, rr)
    YT, _ = oracle.spmm(cols, rows, cr[0], rr[0], lmT["lmap_r"], lmT["R"], vals, A, 0, 5)
    Bloc = B[lmT["gmap_r"] - cr[0]].astype(np.float64)
    np.testing.assert_allclose((Aloc * Y).sum(), (Bloc * YT).sum(), rtol=1e-13, atol=1e-13)


def test_zero_value_entry_propagates_nan():
    """A stored zero is still a task: 0 * inf is NaN in IEEE arithmetic."""
    A = np.array([[np.inf, 1.0]], np.float32)
    B = np.array([[1.0, 1.0]], np.float32)
    out, _ = oracle.sddmm([0], [0], 0, 0, np.array([0.0], np.float32), A, B, 0, 2)
    assert np.isnan(out[0])


# --------------------------------------------------------------- attention

def _attn_instance(seed, n=40, nnz=160, K=5):
    rows, cols, _, _, _, rr, cr = _tiny_problem(seed, M=n, N=n, K=K, nnz=nnz, lo=(0, 0))
    lm = oracle.relabel(rows, cols, rr, cr)
    rng = np.random.default_rng(seed + 100)
    Q = rng.standard_normal((lm["R"], K))
    Kf = rng.standard_normal((lm["C"], K))
    V = rng.standard_normal((lm["C"], K))
    return lm, Q, Kf, V


def test_attention_matches_torch_dense_masked():
    import torch
    lm, Q, Kf, V = _attn_instance(9)
    e, alpha, out = oracle.attention_fwd(lm["rowptr"], lm["colidx"], Q, Kf, V)
    R, C = lm["R"], lm["C"]
    lr = np.repeat(np.arange(R), np.diff(lm["rowptr"]))
    mask = np.zeros((R, C), bool)
    mask[lr, lm["colidx"]] = True
    tq = torch.tensor(Q, requires_grad=True)
    tk = torch.tensor(Kf, requires_grad=True)
    tv = torch.tensor(V, requires_grad=True)
    scores = (tq @ tk.T).masked_fill(~torch.from_numpy(mask), float("-inf"))
    att = torch.softmax(scores, dim=1)
    o = att @ tv
    np.testing.assert_allclose(out, o.detach().numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(alpha, att.detach().numpy()[lr, lm["colidx"]], rtol=1e-12)
    np.testing.assert_allclose(np.bincount(lr, alpha), np.ones(R), rtol=1e-13)
    dout = np.random.default_rng(1).standard_normal(out.shape)
    o.backward(torch.tensor(dout))
    de, dQ, dKf, dV = oracle.attention_bwd(lm["rowptr"], lm["colidx"], Q, Kf, V, alpha, dout)
    np.testing.assert_allclose(dQ, tq.grad.numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(dKf, tk.grad.numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(dV, tv.grad.numpy(), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(np.bincount(lr, de, minlength=R), 0, atol=1e-12)


def test_attention_backward_finite_differences():
    lm, Q, Kf, V = _attn_instance(10, n=12, nnz=40, K=3)
    rng = np.random.default_rng(3)
    W = rng.standard_normal((lm["R"], 3))

    def loss(q, k, v):
        return float((oracle.attention_fwd(lm["rowptr"], lm["colidx"], q, k, v)[2] * W).sum())

    _, alpha, _ = oracle.attention_fwd(lm["rowptr"], lm["colidx"], Q, Kf, V)
    _, dQ, dKf, dV = oracle.attention_bwd(lm["rowptr"], lm["colidx"], Q, Kf, V, alpha, W)
    h = 1e-6
    for X, G, which in ((Q, dQ, 0), (Kf, dKf, 1), (V, dV, 2)):
        num = np.zeros_like(X)
        for idx in np.ndindex(*X.shape):
            args_p = [Q.copy(), Kf.copy(), V.copy()]
            args_m = [Q.copy(), Kf.copy(), V.copy()]
            args_p[which][idx] += h
            args_m[which][idx] -= h
            num[idx] = (loss(*args_p) - loss(*args_m)) / (2 * h)
        np.testing.assert_allclose(G, num, rtol=1e-6, atol=1e-8)


def test_sddmm_spmm_gradients_by_finite_differences():
    """The chain-rule identities the backward relies on, pinned by central
    differences of the oracle forward: d/dA sum(W o SDDMM(S,A,B)) = SpMM(S o W, B)
    and d/dB sum(W2 o SpMM(S,B)) = SpMM^T(S, W2)."""
    rows, cols, vals, A, B, rr, cr = _tiny_problem(21, M=9, N=7, K=3, nnz=25)
    A = A.astype(np.float64).astype(np.float32)
    lm = oracle.relabel(rows, cols, rr, cr)
    lmT = oracle.relabel(cols, rows, cr, rr)
    rng = np.random.default_rng(4)
    W = rng.standard_normal(rows.size)
    W2 = rng.standard_normal((lm["R"], 3))
    h = 1e-3   # loss is linear in A and B: central differences are exact up to rounding

    def f_sddmm(Ax):
        return float((oracle.sddmm(rows, cols, rr[0], cr[0], vals, Ax, B, 0, 3)[0] * W).sum())

    want, _ = oracle.spmm(rows, cols, rr[0], cr[0], lm["lmap_r"], lm["R"],
                          (vals * W).astype(np.float32), B, 0, 3)
    for i, g in enumerate(lm["gmap_r"]):
        for k in range(3):
            Ap, Am = A.copy(), A.copy()
            Ap[g - rr[0], k] += h
            Am[g - rr[0], k] -= h
            fd = (f_sddmm(Ap) - f_sddmm(Am)) / (2 * h)
            assert abs(fd - want[i, k]) <= 1e-4 * (1 + abs(want[i, k]))

    def f_spmm(Bx):
        y, _ = oracle.spmm(rows, cols, rr[0], cr[0], lm["lmap_r"], lm["R"], vals, Bx, 0, 3)
        return float((y * W2).sum())

    W2full = np.zeros((rr[1] - rr[0], 3), np.float32)
    W2full[lm["gmap_r"] - rr[0]] = W2
    wantB, _ = oracle.spmm(cols, rows, cr[0], rr[0], lmT["lmap_r"], lmT["R"], vals, W2full, 0, 3)
    for j, g in enumerate(lmT["gmap_r"]):
        for k in range(3):
            Bp, Bm = B.copy(), B.copy()
            Bp[g - cr[0], k] += h
            Bm[g - cr[0], k] -= h
            fd = (f_spmm(Bp) - f_spmm(Bm)) / (2 * h)
            assert abs(fd - wantB[j, k]) <= 1e-4 * (1 + abs(wantB[j, k]))
