"""The fused attention forward (scores, row softmax and aggregation in one
pass) against the FP64 oracle's masked attention, across K-slice widths,
FP32 and bfloat16, every explicit variant, and patterns whose rows cross lane
groups and work items (R-MAT hub rows, one very long row, single-entry rows,
a block smaller than one work item); the stored row (max, sum) pairs; and
alpha rebuilt from them.

Tolerance.  Each score carries the error of a length-kz FP32 dot product,
|de_p| <= gamma_kz * Me_p with Me_p = sum_k |q_k k_k| and gamma_kz ~ kz u;
an error de in a score perturbs its weight by a relative de, so an output
row satisfies |out - out*| <= (2e-5 + 2 kz u max_p Me_p) * M with M =
sum_p alpha_p |v_p| (the 2e-5 covers the exponentials, the rescalings and
the sums, as in the unfused layer's tests).
"""
import sys

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
U = 2.0 ** -24


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _patterns():
    """(name, rows, cols, n): global ids in [0, n) for both axes."""
    out = []
    p = synth.small_rmat(13, 12, 8, 61)
    out.append(("rmat13", p.rows, p.cols, 1 << 13))
    r, c = synth.uniform_block(700, 900, 3000, 62)
    out.append(("uniform-ragged", r, c, 900))
    # one row of 5000 entries among short rows: spans many work items
    r2, c2 = synth.uniform_block(64, 6000, 600, 63)
    long_c = np.arange(0, 6000, 6000 // 5000, dtype=np.int64)[:5000]
    rows = np.concatenate([r2, np.full(5000, 70, np.int64)])
    cols = np.concatenate([c2, long_c])
    out.append(("one-long-row", rows, cols, 6000))
    # every row a single entry
    idx = np.arange(3000, dtype=np.int64)
    out.append(("diagonal", idx, (idx * 7) % 3000, 3000))
    # fewer entries than one work item
    r3, c3 = synth.uniform_block(20, 20, 37, 64)
    out.append(("tiny", r3, c3, 20))
    return out


def _oracle_case(ref, Q, Kf, V):
    rowptr, colidx = ref["rowptr"], ref["colidx"]
    Qd, Kd, Vd = (x.astype(np.float64) for x in (Q, Kf, V))
    e, alpha, o = oracle.attention_fwd(rowptr, colidx, Qd, Kd, Vd)
    R = Q.shape[0]
    lr = np.repeat(np.arange(R), np.diff(rowptr))
    Me = (np.abs(Qd[lr]) * np.abs(Kd[colidx])).sum(1)
    Mrow = np.zeros(R)
    np.maximum.at(Mrow, lr, Me)
    M_out = np.zeros_like(Qd)
    np.add.at(M_out, lr, alpha[:, None] * np.abs(Vd[colidx]))
    m = np.full(R, -np.inf)
    np.maximum.at(m, lr, e)
    s = np.zeros(R)
    np.add.at(s, lr, np.exp(e - m[lr]))
    return dict(e=e, alpha=alpha, out=o, M_out=M_out, Mrow=Mrow, m=m, s=s, lr=lr)


def _check(spc, plan, ref, Q, Kf, V, kz, dt, variant, what, rounded=None):
    tq, tk, tv = (torch.from_numpy(x).to(DEV) for x in (Q, Kf, V))
    if dt == torch.bfloat16:
        tq, tk, tv = (t.to(torch.bfloat16) for t in (tq, tk, tv))
    out, stats = spc.attention_fwd(plan, tq, tk, tv, kz, variant=variant)
    src = rounded if rounded is not None else (Q, Kf, V)
    o = _oracle_case(ref, *src)
    tol_row = 2e-5 + 2 * kz * U * o["Mrow"]
    assert_within_mag(_np(out), o["out"], o["M_out"] * tol_row[:, None] / 1e-5, 1e-5,
                      f"{what} out")
    st = _np(stats).astype(np.float64)
    dm = 2 * kz * U * o["Mrow"] + 1e-6 * np.abs(o["m"])
    assert np.all(np.abs(st[:, 0] - o["m"]) <= dm), f"{what} row max"
    assert np.all(np.abs(st[:, 1] - o["s"]) <= o["s"] * (2e-5 + 4 * kz * U * o["Mrow"])), \
        f"{what} row sum"
    return out, stats, o


@pytest.mark.parametrize("kz", [16, 32, 64, 128])
def test_fused_attention_fp32_against_oracle(kz):
    spc = _spc()
    for name, rows, cols, n in _patterns():
        _say(f"fused attention fp32 kz={kz} {name} nnz={rows.size}")
        plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV),
                                   torch.from_numpy(cols).to(DEV), (0, n), (0, n))
        ref = oracle.relabel(rows, cols, (0, n), (0, n))
        R, C = plan.R, plan.C
        Q = synth.dense_f32(71, 0, R, kz)
        Kf = synth.dense_f32(72, 0, C, kz)
        V = synth.dense_f32(73, 0, C, kz)
        nvec = kz // 4
        variants = [-1] + [lg | (lgs << 4) for lg in (2, 3, 4) for lgs in (4, 5, 6)
                           if nvec % (1 << lg) == 0 and nvec // (1 << lg) in (1, 2)]
        for v in variants:
            out, stats, o = _check(spc, plan, ref, Q, Kf, V, kz, torch.float32, v,
                                   f"fp32 kz={kz} {name} v={v}")
        # alpha rebuilt from the stored pairs and recomputed scores
        e = spc.sddmm(plan, None, torch.from_numpy(Q).to(DEV), torch.from_numpy(Kf).to(DEV), kz)
        alpha = _np(spc.row_softmax_apply(plan, e, stats))
        tol = 2e-5 + 4 * kz * U * o["Mrow"][o["lr"]]
        assert np.all(np.abs(alpha - o["alpha"]) <= tol * np.maximum(o["alpha"], 1e-30) + 1e-7), \
            f"alpha from stats kz={kz} {name}"


@pytest.mark.parametrize("kz", [32, 64])
def test_fused_attention_bf16_against_oracle_on_rounded_inputs(kz):
    spc = _spc()
    name, rows, cols, n = _patterns()[0]
    _say(f"fused attention bf16 kz={kz} {name}")
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               (0, n), (0, n))
    ref = oracle.relabel(rows, cols, (0, n), (0, n))
    Q = synth.dense_f32(81, 0, plan.R, kz)
    Kf = synth.dense_f32(82, 0, plan.C, kz)
    V = synth.dense_f32(83, 0, plan.C, kz)
    rnd = tuple(oracle.bf16_to_f32(oracle.bf16_rne(x)) for x in (Q, Kf, V))
    nvec = kz // 8   # 16-byte vectors of bfloat16 per row
    for v in (-1, (nvec.bit_length() - 1) | (5 << 4)):
        _check(spc, plan, ref, Q, Kf, V, kz, torch.bfloat16, v, f"bf16 kz={kz} v={v}",
               rounded=rnd)


def test_fused_attention_matches_unfused_layer_and_rejects_uncovered_shapes():
    spc = _spc()
    from paper_2404_19638_amd import autograd as ag
    name, rows, cols, n = _patterns()[0]
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               (0, n), (0, n), spc.BUILD_CSC)
    kz = 32
    tq, tk, tv = (torch.from_numpy(synth.dense_f32(s, 0, m, kz)).to(DEV)
                  for s, m in ((91, plan.R), (92, plan.C), (93, plan.C)))
    a = ag.gnn_attention(plan, tq, tk, tv, fused=True)
    b = ag.gnn_attention(plan, tq, tk, tv, fused=False)
    assert float((a - b).abs().max()) <= 1e-4 * float(b.abs().max())
    for bad_kz in (8, 12, 48):
        assert not spc.attention_supported(bad_kz)
        q = torch.zeros((plan.R, bad_kz), device=DEV)
        k = torch.zeros((plan.C, bad_kz), device=DEV)
        with pytest.raises(spc.Spc3dError):
            spc.attention_fwd(plan, q, k, k, bad_kz)


def test_automatic_forward_choice_runs_the_chosen_kernels():
    """gnn_attention with fused left open: for inference with bfloat16 (and
    small FP32) operands its output is the one-pass kernel's, bit for bit;
    with a gradient to record it is the three kernels'."""
    spc = _spc()
    from paper_2404_19638_amd import autograd as ag
    name, rows, cols, n = _patterns()[0]
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               (0, n), (0, n), spc.BUILD_CSC)
    _say(f"automatic attention forward {name} nnz={plan.nnz}")
    kz = 32
    for dt in (torch.bfloat16, torch.float32):
        tq, tk, tv = (torch.from_numpy(synth.dense_f32(s, 0, m, kz)).to(DEV).to(dt)
                      for s, m in ((94, plan.R), (95, plan.C), (96, plan.C)))
        with torch.no_grad():
            auto = ag.gnn_attention(plan, tq, tk, tv)
            one = ag.gnn_attention(plan, tq, tk, tv, fused=True)
            three = ag.gnn_attention(plan, tq, tk, tv, fused=False)
        assert torch.equal(auto.view(torch.int16 if dt == torch.bfloat16 else torch.int32),
                           one.view(torch.int16 if dt == torch.bfloat16 else torch.int32))
        tqg = tq.clone().requires_grad_()
        auto_g = ag.gnn_attention(plan, tqg, tk, tv)
        assert torch.equal(auto_g.detach().view(torch.int16 if dt == torch.bfloat16 else torch.int32),
                           three.view(torch.int16 if dt == torch.bfloat16 else torch.int32))


def test_row_softmax_and_backward_against_oracle():
    """The separate softmax kernels (forward and backward) on the same patterns,
    with 16-byte aligned arrays and with arrays offset by one float (the
    scalar-load path)."""
    spc = _spc()
    kz = 16
    for name, rows, cols, n in _patterns():
        _say(f"row softmax {name} nnz={rows.size}")
        plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV),
                                   torch.from_numpy(cols).to(DEV), (0, n), (0, n))
        ref = oracle.relabel(rows, cols, (0, n), (0, n))
        R, C, nnz = plan.R, plan.C, plan.nnz
        Q = synth.dense_f32(101, 0, R, kz)
        Kf = synth.dense_f32(102, 0, C, kz)
        V = synth.dense_f32(103, 0, C, kz)
        W = synth.dense_f32(104, 0, R, kz)
        o = _oracle_case(ref, Q, Kf, V)
        Qd, Kd, Vd, Wd = (x.astype(np.float64) for x in (Q, Kf, V, W))
        de_ref, _, _, _ = oracle.attention_bwd(ref["rowptr"], ref["colidx"], Qd, Kd, Vd,
                                               o["alpha"], Wd)
        tq, tk, tv, tw = (torch.from_numpy(x).to(DEV) for x in (Q, Kf, V, W))
        tol = 2e-5 + 4 * kz * U * o["Mrow"][o["lr"]]
        for off in (0, 1):
            e = torch.empty(nnz + off, device=DEV)[off:]
            spc.sddmm(plan, None, tq, tk, kz, out=e)
            a_buf = torch.empty(nnz + off, device=DEV)[off:]
            alpha = spc.row_softmax(plan, e, out=a_buf)
            ga = _np(alpha)
            assert np.all(np.abs(ga - o["alpha"]) <= tol * np.maximum(o["alpha"], 1e-30) + 1e-7), \
                f"softmax {name} offset={off}"
            da = torch.empty(nnz + off, device=DEV)[off:]
            spc.sddmm(plan, None, tw, tv, kz, out=da)
            de = _np(spc.row_softmax_bwd(plan, alpha, da))
            # |de_p| pieces: alpha_p |dalpha_p| and alpha_p sum_q alpha_q |dalpha_q|
            lr, colidx = o["lr"], ref["colidx"]
            dal = (np.abs(Wd[lr]) * np.abs(Vd[colidx])).sum(1)
            rs = np.bincount(lr, o["alpha"] * dal, minlength=R)
            M_de = o["alpha"] * (dal + rs[lr])
            assert_within_mag(de, de_ref, M_de * (tol / 1e-5), 1e-5, f"softmax bwd {name} off={off}")
