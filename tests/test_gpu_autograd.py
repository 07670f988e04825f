"""Hand-written backward (torch.autograd.Function over libspc3d) against the
FP64 oracle: its analytic backward, and central finite differences of its
forward, on the 256-vertex / 2,000-entry instance with K = 8; SDDMM / SpMM /
gather gradients with sampling values; and the attention workload (R-MAT
2^20 vertices, average degree 32, K = 64) on sampled rows, with timings.

Tolerances.  Forward and gradient entries are sums of products; each GPU
value carries a few FP32 roundings per term (exp, division, products, sums
of depth well under 100), so |g - g*| <= 2e-5 * M with M the sum of the
magnitudes of the terms, computed from the oracle's own intermediates.
"""
import json
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth
from helpers import assert_within_mag

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"
TOL = 2e-5


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _mods():
    from paper_2404_19638_amd import autograd as ag
    from paper_2404_19638_amd import spc3d as spc
    return spc, ag


def _np(t):
    return t.detach().cpu().numpy()


def _attention_magnitudes(rowptr, colidx, Q, Kf, V, alpha, dout, de):
    """Magnitude sums M for out, dQ, dKf, dV from the oracle's intermediates."""
    R, C = Q.shape[0], Kf.shape[0]
    lr = np.repeat(np.arange(R), np.diff(rowptr))
    aV = np.abs(V)
    dal = (np.abs(dout[lr]) * aV[colidx]).sum(1)          # bounds |dalpha_p|
    rowsum = np.bincount(lr, alpha * dal, minlength=R)
    dem = alpha * (dal + rowsum[lr]) + np.abs(de)         # bound on |de_p| and its pieces
    M_out = np.zeros_like(Q)
    np.add.at(M_out, lr, alpha[:, None] * aV[colidx])
    M_dQ = np.zeros_like(Q)
    np.add.at(M_dQ, lr, dem[:, None] * np.abs(Kf)[colidx])
    M_dK = np.zeros_like(Kf)
    np.add.at(M_dK, colidx, dem[:, None] * np.abs(Q)[lr])
    M_dV = np.zeros_like(V)
    np.add.at(M_dV, colidx, alpha[:, None] * np.abs(dout)[lr])
    return M_out, M_dQ, M_dK, M_dV


def _attention_magnitudes_sparse(rowptr, colidx, Q, Kf, V, alpha, dout, de, chunk=1 << 20):
    """_attention_magnitudes for millions of entries: the per-entry bound of
    |dalpha_p| in chunks, the row and column sums as sparse products."""
    import scipy.sparse as sps
    R, C = Q.shape[0], Kf.shape[0]
    nnz = colidx.shape[0]
    lr = np.repeat(np.arange(R, dtype=np.int64), np.diff(rowptr))
    aW, aV = np.abs(dout), np.abs(V)
    dal = np.empty(nnz)
    for s in range(0, nnz, chunk):
        t = min(s + chunk, nnz)
        dal[s:t] = np.einsum("ij,ij->i", aW[lr[s:t]], aV[colidx[s:t]])
    rowsum = np.bincount(lr, alpha * dal, minlength=R)
    dem = alpha * (dal + rowsum[lr]) + np.abs(de)
    del dal, rowsum, lr
    S_a = sps.csr_matrix((alpha, colidx, rowptr), shape=(R, C))
    S_d = sps.csr_matrix((dem, colidx, rowptr), shape=(R, C))
    return (S_a @ aV, S_d @ np.abs(Kf), (S_d.T @ np.abs(Q)), (S_a.T @ aW))


@pytest.mark.parametrize("K,fused", [(8, False), (16, True)])
def test_attention_backward_fd_instance(K, fused):
    """K = 8: the three-kernel layer; K = 16: the fused forward, whose backward
    recomputes the scores and rebuilds alpha from the stored row statistics."""
    spc, ag = _mods()
    n, nnz = 256, 2000
    rows, cols = synth.uniform_block(n, n, nnz, 4242)
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               (0, n), (0, n), spc.BUILD_CSC)
    ref = oracle.relabel(rows, cols, (0, n), (0, n))
    R, C = plan.R, plan.C
    Q = synth.dense_f32(11, 0, R, K)
    Kf = synth.dense_f32(12, 0, C, K)
    V = synth.dense_f32(13, 0, C, K)
    W = synth.dense_f32(14, 0, R, K)
    tq = torch.from_numpy(Q).to(DEV).requires_grad_()
    tk = torch.from_numpy(Kf).to(DEV).requires_grad_()
    tv = torch.from_numpy(V).to(DEV).requires_grad_()
    out = ag.gnn_attention(plan, tq, tk, tv, fused=fused)
    (out * torch.from_numpy(W).to(DEV)).sum().backward()
    Qd, Kd, Vd, Wd = (x.astype(np.float64) for x in (Q, Kf, V, W))
    e, alpha, o = oracle.attention_fwd(ref["rowptr"], ref["colidx"], Qd, Kd, Vd)
    de, dQ, dK, dV = oracle.attention_bwd(ref["rowptr"], ref["colidx"], Qd, Kd, Vd, alpha, Wd)
    M_out, M_dQ, M_dK, M_dV = _attention_magnitudes(ref["rowptr"], ref["colidx"], Qd, Kd, Vd,
                                                    alpha, Wd, de)
    assert_within_mag(_np(out), o, M_out, TOL, "attention out")
    assert_within_mag(_np(tq.grad), dQ, M_dQ, TOL, "dQ")
    assert_within_mag(_np(tk.grad), dK, M_dK, TOL, "dKf")
    assert_within_mag(_np(tv.grad), dV, M_dV, TOL, "dV")

    # central finite differences of the FP64 oracle forward at sampled coordinates
    def loss(q, k, v):
        return float((oracle.attention_fwd(ref["rowptr"], ref["colidx"], q, k, v)[2] * Wd).sum())

    rng = np.random.default_rng(5)
    h = 1e-6
    for X, G, which in ((Qd, tq.grad, 0), (Kd, tk.grad, 1), (Vd, tv.grad, 2)):
        g = _np(G)
        scale = np.abs(g).max()
        for _ in range(25):
            idx = (int(rng.integers(X.shape[0])), int(rng.integers(X.shape[1])))
            args_p = [Qd.copy(), Kd.copy(), Vd.copy()]
            args_m = [Qd.copy(), Kd.copy(), Vd.copy()]
            args_p[which][idx] += h
            args_m[which][idx] -= h
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            assert abs(g[idx] - fd) <= 1e-4 * scale, (which, idx, g[idx], fd)


def test_sddmm_spmm_gather_gradients_with_values():
    spc, ag = _mods()
    p = synth.small_rmat(11, 8, 16, 99, row_range=(1 << 10, 1 << 11), col_range=(0, 1 << 10))
    k0, kz = 4, 8
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range, spc.BUILD_CSC)
    ref = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range)
    perm = ref["perm"]
    As = torch.from_numpy(p.A_src).to(DEV).requires_grad_()
    Bs = torch.from_numpy(p.B_src).to(DEV).requires_grad_()
    vals = torch.from_numpy(p.vals[perm]).to(DEV).requires_grad_()
    W1 = synth.uniform_f32(501, plan.nnz)           # weights of the SDDMM output (slot order)
    W2 = synth.dense_f32(502, 0, plan.R, kz)        # weights of the SpMM output
    A = ag.gather(plan, spc.ROWS, As, k0, kz)
    B = ag.gather(plan, spc.COLS, Bs, k0, kz)
    c = ag.sddmm(plan, vals, A, B)
    y = ag.spmm(plan, vals, B, 0)
    loss = (c * torch.from_numpy(W1).to(DEV)).sum() + (y * torch.from_numpy(W2).to(DEV)).sum()
    loss.backward()
    # chain rule written out with the oracle (caller order): let w1 be W1 in caller order
    w1 = np.empty(plan.nnz, np.float32)
    w1[perm] = W1
    ro, co, lo_r, lo_c = p.rows, p.cols, p.row_range[0], p.col_range[0]
    dot, mdot = oracle.sddmm(ro, co, lo_r, lo_c, None, p.A_src, p.B_src, k0, kz)
    # d vals_p = W1_p <a,b> + <W2_row, b>
    lmap_r = ref["lmap_r"]
    w2dot = (W2.astype(np.float64)[lmap_r[ro - lo_r]] *
             p.B_src.astype(np.float64)[co - lo_c, k0:k0 + kz]).sum(1)
    want_dv = w1 * dot + w2dot
    mag_dv = np.abs(w1) * mdot + (np.abs(W2.astype(np.float64)[lmap_r[ro - lo_r]]) *
                                  np.abs(p.B_src[co - lo_c, k0:k0 + kz])).sum(1)
    assert_within_mag(_np(vals.grad)[np.argsort(perm)], want_dv, mag_dv, TOL, "dvals")
    # dA_src rows: SpMM of (W1 o s) with B, scattered into the K-slice
    sw = (w1 * p.vals).astype(np.float32)
    ya, ma = oracle.spmm(ro, co, lo_r, lo_c, lmap_r, ref["R"], sw, p.B_src, k0, kz)
    gA = _np(As.grad)
    assert np.all(gA[:, :k0] == 0) and np.all(gA[:, k0 + kz:] == 0)
    assert_within_mag(gA[ref["gmap_r"] - lo_r, k0:k0 + kz], ya, ma, TOL, "dA_src")
    # dB_src: SpMM^T of (W1 o s) with A plus SpMM^T of s with W2
    lmap_c = ref["lmap_c"]
    yb1, mb1 = oracle.spmm(co, ro, lo_c, lo_r, lmap_c, ref["C"], sw, p.A_src, k0, kz)
    W2full = np.zeros_like(p.A_src)
    W2full[ref["gmap_r"] - lo_r, k0:k0 + kz] = W2
    yb2, mb2 = oracle.spmm(co, ro, lo_c, lo_r, lmap_c, ref["C"], p.vals, W2full, k0, kz)
    gB = _np(Bs.grad)
    assert_within_mag(gB[ref["gmap_c"] - lo_c, k0:k0 + kz], yb1 + yb2, mb1 + mb2, TOL, "dB_src")


def test_attention_workload_full_size():
    """R-MAT 2^20, degree 32, K = 64: forward + backward on the GPU, the output
    (three-kernel and fused forward), dQ, dKf and dV compared with the FP64
    oracle element by element at full size, forward/backward timings."""
    spc, ag = _mods()
    p = synth.attention(dense=False)
    K = 64
    _say(f"attention workload nnz={p.nnz}")
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range, spc.BUILD_CSC)
    R, C = plan.R, plan.C
    Q = synth.dense_f32(21, 0, R, K)
    Kf = synth.dense_f32(22, 0, C, K)
    V = synth.dense_f32(23, 0, C, K)
    W = synth.dense_f32(24, 0, R, K)
    tq = torch.from_numpy(Q).to(DEV).requires_grad_()
    tk = torch.from_numpy(Kf).to(DEV).requires_grad_()
    tv = torch.from_numpy(V).to(DEV).requires_grad_()
    tw = torch.from_numpy(W).to(DEV)
    for _ in range(2):   # warm-up
        out = ag.gnn_attention(plan, tq, tk, tv)
        (out * tw).sum().backward()
        tq.grad = tk.grad = tv.grad = None
    with torch.no_grad():
        # forward of the one-pass kernel, for comparison with the three-kernel layer
        ag.gnn_attention(plan, tq, tk, tv, fused=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            out_fused = ag.gnn_attention(plan, tq, tk, tv, fused=True)
        torch.cuda.synchronize()
        t_fused = (time.perf_counter() - t0) / 5
    torch.cuda.synchronize()
    reps = 5
    t_f = t_b = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        out = ag.gnn_attention(plan, tq, tk, tv)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (out * tw).sum().backward()
        torch.cuda.synchronize()
        t_f += t1 - t0
        t_b += time.perf_counter() - t1
        if _ < reps - 1:
            tq.grad = tk.grad = tv.grad = None
    m = plan.maps()
    rowptr, colidx = _np(m["rowptr"]), _np(m["colidx"])
    got = {"out": _np(out), "fused out": _np(out_fused), "dQ": _np(tq.grad),
           "dKf": _np(tk.grad), "dV": _np(tv.grad)}
    # every row and column, the longest included (about 64,500 entries each),
    # against the FP64 oracle at full size (tens of seconds on one host core)
    _say("attention workload: FP64 oracle forward and backward at full size")
    Qd, Kd, Vd, Wd = (x.astype(np.float64) for x in (Q, Kf, V, W))
    e, alpha, o = oracle.attention_fwd(rowptr, colidx, Qd, Kd, Vd)
    de, dQ, dK, dV = oracle.attention_bwd(rowptr, colidx, Qd, Kd, Vd, alpha, Wd)
    del e
    M_out, M_dQ, M_dK, M_dV = _attention_magnitudes_sparse(rowptr, colidx, Qd, Kd, Vd, alpha,
                                                           Wd, de)
    lens_r, lens_c = np.diff(rowptr), np.bincount(colidx, minlength=C)
    _say(f"  longest row {lens_r.max()}, longest column {lens_c.max()}")
    assert_within_mag(got["out"], o, M_out, TOL, "attention out (full size)")
    assert_within_mag(got["fused out"], o, M_out, TOL, "fused out (full size)")
    assert_within_mag(got["dQ"], dQ, M_dQ, TOL, "dQ (full size)")
    assert_within_mag(got["dKf"], dK, M_dK, TOL, "dKf (full size)")
    assert_within_mag(got["dV"], dV, M_dV, TOL, "dV (full size)")
    del Qd, Kd, Vd, Wd, alpha, o, de, dQ, dK, dV, M_out, M_dQ, M_dK, M_dV, got
    # the same layer with bfloat16 Q, Kf, V (mixed precision), timed the same way
    bq, bk, bv = (t.detach().bfloat16().requires_grad_() for t in (tq, tk, tv))
    for _ in range(2):
        (ag.gnn_attention(plan, bq, bk, bv) * tw).sum().backward()
    torch.cuda.synchronize()
    b_f = b_b = 0.0
    for _ in range(reps):
        bq.grad = bk.grad = bv.grad = None
        t0 = time.perf_counter()
        out_b = ag.gnn_attention(plan, bq, bk, bv)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        (out_b * tw).sum().backward()
        torch.cuda.synchronize()
        b_f += t1 - t0
        b_b += time.perf_counter() - t1
    with torch.no_grad():
        ag.gnn_attention(plan, bq, bk, bv, fused=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ag.gnn_attention(plan, bq, bk, bv, fused=True)
        torch.cuda.synchronize()
        b_fused = (time.perf_counter() - t0) / reps
    flops = 2 * 2 * K * p.nnz
    print("ATTENTION_REPORT " + json.dumps({
        "workload": "rmat20-deg32-whole-K64", "nnz": p.nnz, "R": R, "C": C,
        "forward": "three kernels (SDDMM, row softmax, SpMM)",
        "forward_ms": round(t_f / reps * 1e3, 3), "backward_ms": round(t_b / reps * 1e3, 3),
        "forward_ms_fused_no_grad": round(t_fused * 1e3, 3),
        "bf16_forward_ms": round(b_f / reps * 1e3, 3), "bf16_backward_ms": round(b_b / reps * 1e3, 3),
        "bf16_forward_ms_fused_no_grad": round(b_fused * 1e3, 3),
        "forward_sddmm_spmm_GFLOPs": round(flops / (t_f / reps) / 1e9, 1)}), flush=True)


@pytest.mark.parametrize("fused", [False, True])
def test_bf16_attention_training_against_fp32_on_rounded_inputs(fused):
    """Graph attention with bfloat16 Q, Kf and V (mixed precision: FP32
    accumulation, the output gradient rounded to bfloat16 where an SDDMM meets
    bfloat16 operands, gradients returned in bfloat16).  Against the FP64
    oracle on the rounded inputs (and rounded output gradient): the forward
    within 2e-5 M, every gradient within 2e-5 M plus one bfloat16 rounding.
    Beside it, against the FP32 layer on the same inputs: the forward within
    1e-5 of the magnitude of its terms, every gradient within 2^-6 of the FP32
    layer's largest gradient entry (one bfloat16 rounding of dOut and one of
    the result)."""
    spc, ag = _mods()
    p = synth.small_rmat(11, 8, 64, 77, row_range=(1 << 10, 1 << 11), col_range=(0, 1 << 10))
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range, spc.BUILD_CSC)
    g = torch.Generator().manual_seed(11)
    Qb = torch.randn((plan.R, 32), generator=g).to(DEV).bfloat16()
    Kb = torch.randn((plan.C, 32), generator=g).to(DEV).bfloat16()
    Vb = torch.randn((plan.C, 32), generator=g).to(DEV).bfloat16()
    G = torch.randn((plan.R, 32), generator=g).to(DEV)
    _say(f"bf16 attention fused={fused} nnz={plan.nnz}")
    outs, grads = [], []
    for dt in (torch.bfloat16, torch.float32):
        ts = [t.to(dt).clone().requires_grad_() for t in (Qb, Kb, Vb)]
        out = ag.gnn_attention(plan, *ts, fused=fused)
        torch.autograd.backward(out, G)
        assert all(t.grad.dtype == dt for t in ts)
        outs.append(out.detach().float())
        grads.append([t.grad.float() for t in ts])
    # forward: the same products of bfloat16 values, accumulated in FP32
    ref = outs[1]
    assert (outs[0] - ref).abs().max().item() <= 1e-5 * (ref.abs().max().item() + 1.0)
    for name, gb, gf in zip(("dQ", "dKf", "dV"), grads[0], grads[1]):
        bound = 2.0 ** -6 * gf.abs().max().item()
        err = (gb - gf).abs().max().item()
        _say(f"  {name}: max |bf16 - fp32| {err:.3e} (bound {bound:.3e})")
        assert err <= bound, (name, err, bound)
    # Against the FP64 oracle on the same rounded values: Q, Kf, V as stored in
    # bfloat16 and the output gradient rounded to bfloat16 as the backward
    # rounds it before its SDDMM and transposed SpMM.  The forward (FP32 out)
    # meets the FP32 bar; each returned gradient is that bar plus its own
    # rounding to bfloat16 (unit roundoff 2^-8).
    m = plan.maps()
    rowptr, colidx = _np(m["rowptr"]), _np(m["colidx"])
    Qd, Kd, Vd = (t.float().cpu().numpy().astype(np.float64) for t in (Qb, Kb, Vb))
    Gd = G.bfloat16().float().cpu().numpy().astype(np.float64)
    _, alpha, o = oracle.attention_fwd(rowptr, colidx, Qd, Kd, Vd)
    de, dQ, dK, dV = oracle.attention_bwd(rowptr, colidx, Qd, Kd, Vd, alpha, Gd)
    Ms = _attention_magnitudes(rowptr, colidx, Qd, Kd, Vd, alpha, Gd, de)
    assert_within_mag(_np(outs[0]), o, Ms[0], TOL, "bf16 attention out vs oracle")
    for name, gb, want, M in zip(("dQ", "dKf", "dV"), grads[0], (dQ, dK, dV), Ms[1:]):
        gb = _np(gb).astype(np.float64)
        bound = TOL * M + 2.0 ** -8 * (np.abs(want) + TOL * M) + 1e-37
        err = np.abs(gb - want)
        _say(f"  {name} vs oracle: max err/bound {float((err / bound).max()):.3f}")
        assert (err <= bound).all(), (name, int((err > bound).sum()))


def test_column_sliced_inputs_in_forward_and_backward():
    """Operands that are column blocks of wider tensors (not contiguous): the
    functions pack them once and keep the packed copies for the backward, so
    the forward equals that of the same values given contiguous bit for bit,
    and the gradients up to the order in which autograd adds the
    contributions of an operand's several uses (SDDMM and SpMM with values,
    and the attention layer)."""
    spc, ag = _mods()
    p = synth.small_rmat(11, 8, 16, 97, row_range=(1 << 10, 1 << 11), col_range=(0, 1 << 10))
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range, spc.BUILD_CSC)
    R, C, K = plan.R, plan.C, 16
    _say(f"column-sliced operands nnz={plan.nnz}")
    wide_r = torch.from_numpy(synth.dense_f32(601, 0, R, 3 * K)).to(DEV)
    wide_c = torch.from_numpy(synth.dense_f32(602, 0, C, 3 * K)).to(DEV)
    vals = torch.from_numpy(synth.uniform_f32(603, plan.nnz)).to(DEV)
    G1 = torch.from_numpy(synth.uniform_f32(604, plan.nnz)).to(DEV)
    G2 = torch.from_numpy(synth.dense_f32(605, 0, R, K)).to(DEV)

    def run(sliced):
        if sliced:
            wr = wide_r.clone().requires_grad_()
            wc = wide_c.clone().requires_grad_()
            A, B, V = wr[:, K:2 * K], wc[:, :K], wc[:, 2 * K:]
            assert not (A.is_contiguous() or B.is_contiguous() or V.is_contiguous())
            leaves = (wr, wc)
        else:
            A = wide_r[:, K:2 * K].contiguous().requires_grad_()
            B = wide_c[:, :K].contiguous().requires_grad_()
            V = wide_c[:, 2 * K:].contiguous().requires_grad_()
            leaves = (A, B, V)
        v = vals.clone().requires_grad_()
        c = ag.sddmm(plan, v, A, B)
        y = ag.spmm(plan, v, B, 0)
        att = ag.gnn_attention(plan, A, B, V)
        ((c * G1).sum() + (y * G2).sum() + (att * G2).sum()).backward()
        if sliced:
            gr, gc = leaves[0].grad, leaves[1].grad
            grads = (gr[:, K:2 * K], gc[:, :K], gc[:, 2 * K:])
        else:
            grads = tuple(t.grad for t in leaves)
        return [c.detach(), y.detach(), att.detach(), v.grad, *grads]

    got, want = run(True), run(False)
    for a, b in zip(got[:3], want[:3]):
        assert torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))
    for a, b in zip(got[3:], want[3:]):
        scale = b.abs().max().item()
        assert (a - b).abs().max().item() <= 1e-6 * scale, (a - b).abs().max().item()
