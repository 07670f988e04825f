"""GPU tests of the learned variant selector: the feature kernel and the MLP
kernels (forward, backward, loss, Adam, masked argmin) through the C ABI
against the FP64 oracle (oracle/mlp.py), a short training run checked against
the oracle's trajectory, and a small end-to-end selector run judged by the
exhaustive autotuner.

Floating-point bar: an FP32 sum of depth d (terms added one after another,
each rounding at most u = 2^-24) lies within (d + 2) u M of the exact value,
M the sum of the magnitudes of its terms; each check below states its d.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2404_19638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # pragma: no cover - collected on CPU hosts too
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"
U = 2.0 ** -24


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _within(got, ref, mag, depth, what):
    bound = (depth + 2) * U * np.asarray(mag) + 1e-30
    err = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64))
    bad = err > bound
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} beyond (d+2)uM, d={depth}; "
                           f"worst err/M {(err / np.maximum(mag, 1e-300)).max():.3e}")


# --------------------------------------------------------------- features

def _feature_cases():
    n = 1 << 12
    long_rows = np.r_[np.zeros(40000, np.int64), np.arange(1, 500)]
    long_cols = np.r_[np.arange(40000), np.zeros(499, np.int64)]
    b0 = synth.selector_block(0, lg_hi=14)
    b1 = synth.selector_block(1, lg_hi=14)
    t = synth.tiny()
    g = synth.small_rmat(12, 8, 32, 5)
    return {
        "tiny": (t.rows, t.cols, (0, n), (0, n)),
        "rmat12": (g.rows, g.cols, (0, n), (0, n)),
        "sel_uniform": (b0["rows"], b0["cols"], (0, b0["n"]), (0, b0["n"])),
        "sel_rmat": (b1["rows"], b1["cols"], (0, b1["n"]), (0, b1["n"])),
        "long_row": (long_rows, long_cols, (0, 500), (0, 40000)),
        "one_entry": (np.array([3]), np.array([7]), (0, 10), (0, 10)),
    }


@pytest.mark.parametrize("name", ["tiny", "rmat12", "sel_uniform", "sel_rmat", "long_row",
                                  "one_entry"])
def test_features_match_oracle(name):
    spc = _spc()
    rows, cols, rr, cr = _feature_cases()[name]
    _say(f"features {name} nnz={len(rows)}")
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               rr, cr, spc.BUILD_CSC)
    for transpose in (0, 1):
        for kz, dt in ((16, spc.F32), (128, spc.BF16), (24, spc.F32)):
            got = _np(spc.plan_features(plan, kz, dt, transpose))
            ref = omlp.features(rows, cols, kz, dt == spc.BF16, transpose=bool(transpose))
            # fractions: the FP64 quotient rounded to FP32 on both sides
            np.testing.assert_array_equal(got[:16], ref[:16].astype(np.float32))
            np.testing.assert_array_equal(got[22], ref[22])
            # logarithms: FP64 log2 on the device rounded to FP32
            np.testing.assert_allclose(got[16:22], ref[16:22], rtol=2 ** -23, atol=1e-7)


def test_features_argument_errors():
    spc = _spc()
    plan = spc.plan_create_coo(torch.tensor([1, 2], device=DEV), torch.tensor([3, 4], device=DEV),
                               (0, 8), (0, 8))
    with pytest.raises(spc.Spc3dError):
        spc.plan_features(plan, 16, spc.F32, transpose=1)   # no CSC view
    with pytest.raises(spc.Spc3dError):
        spc.plan_features(plan, 0, spc.F32)


# ------------------------------------------------------------ dense layers

def _rand(shape, seed, scale=1.0):
    n = int(np.prod(shape))
    return (synth.uniform_f32(seed, n).reshape(shape) * np.float32(scale)).astype(np.float32)


@pytest.mark.parametrize("n,fin,fout", [(1, 23, 64), (33, 64, 64), (100, 64, 60),
                                        (3000, 23, 64), (257, 5, 3)])
@pytest.mark.parametrize("relu", [0, 1])
@pytest.mark.parametrize("bias", [True, False])
def test_linear_fwd_bwd_parity(n, fin, fout, relu, bias):
    spc = _spc()
    _say(f"linear n={n} fin={fin} fout={fout} relu={relu} bias={bias}")
    seed = 1000 + n + 7 * fin + 13 * fout
    X = _rand((n, fin), seed)
    W = _rand((fout, fin), seed + 1, 1 / math.sqrt(fin))
    b = _rand((fout,), seed + 2) if bias else None
    dY = _rand((n, fout), seed + 3)
    tX, tW = torch.from_numpy(X).to(DEV), torch.from_numpy(W).to(DEV)
    tb = torch.from_numpy(b).to(DEV) if bias else None
    Y = spc.mlp_linear_fwd(tX, tW, tb, relu=bool(relu))
    Yg = _np(Y)
    ref = omlp.linear_fwd(X, W, b, relu=False)
    mag = np.abs(X.astype(np.float64)) @ np.abs(W.astype(np.float64)).T
    if bias:
        mag = mag + np.abs(b)
    if relu:
        # where the exact pre-activation is clearly of one sign the ReLU decision
        # is fixed; within the error bound either side is correct
        bound = (fin + 3) * U * mag
        clear = np.abs(ref) > bound
        ref_act = np.where(ref > 0, ref, 0.0)
        _within(Yg[clear], ref_act[clear], mag[clear], fin + 1, "forward (relu)")
        assert np.all((Yg[~clear] == 0) | (np.abs(Yg[~clear] - ref[~clear]) <= bound[~clear]))
    else:
        _within(Yg, ref, mag, fin + 1, "forward")
    # backward from the device's own Y (its ReLU decisions), gradients vs FP64
    tdY = torch.from_numpy(dY).to(DEV)
    dX, dW, db = spc.mlp_linear_bwd(tX, tW, Y, tdY, relu=bool(relu))
    rdX, rdW, rdb = omlp.linear_bwd(X, W, Yg, dY, relu=bool(relu))
    G = np.abs(np.where(Yg > 0, dY, 0.0) if relu else dY.astype(np.float64))
    _within(_np(dX), rdX, G @ np.abs(W.astype(np.float64)), fout, "dX")
    nblk = (n + 31) // 32
    _within(_np(dW), rdW, G.T @ np.abs(X.astype(np.float64)), 32 + nblk, "dW")
    _within(_np(db), rdb, G.sum(axis=0), 32 + nblk, "db")


def test_linear_bwd_zero_rows_clears_gradients():
    spc = _spc()
    X = torch.empty((0, 4), device=DEV)
    W = torch.ones((3, 4), device=DEV)
    dY = torch.empty((0, 3), device=DEV)
    dW = torch.full((3, 4), 7.0, device=DEV)
    db = torch.full((3,), 7.0, device=DEV)
    spc.mlp_linear_bwd(X, W, None, dY, relu=False, need_dx=False, dW=dW, db=db)
    assert not dW.any() and not db.any()


def test_mse_adam_argmin_parity():
    spc = _spc()
    n, m = 700, 60
    P = _rand((n, m), 71)
    T = _rand((n, m), 72)
    M = (synth.uniform_f32(73, n * m).reshape(n, m) > 0).astype(np.float32)
    loss, dP = spc.mlp_mse(torch.from_numpy(P).to(DEV), torch.from_numpy(T).to(DEV),
                           torch.from_numpy(M).to(DEV))
    rl, rdP = omlp.mse(P, T, M)
    c = M.sum()
    d = (P.astype(np.float64) - T) ** 2 * M
    _within([loss.item()], [rl], [d.sum() / c], n * m // 256 + 8 + 2, "loss")
    # dP = (2/c) m (p - t): two roundings of one product chain
    _within(_np(dP), rdP, np.abs(rdP), 4, "dP")

    # Adam: three steps from zero moments.  The C ABI takes the hyperparameters
    # as FP32 arguments, so the oracle is given the same FP32-rounded values.
    lr, b1, b2, eps = (float(np.float32(x)) for x in (1e-2, 0.9, 0.999, 1e-8))
    w = _rand((1000,), 74)
    g = [_rand((1000,), 75 + k) for k in range(3)]
    tw = torch.from_numpy(w).to(DEV)
    tm, tv = torch.zeros(1000, device=DEV), torch.zeros(1000, device=DEV)
    rw, rm, rv = w.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for t in range(1, 4):
        spc.mlp_adam(tw, torch.from_numpy(g[t - 1]).to(DEV), tm, tv, lr, b1, b2, eps, t)
        rw, rm, rv = omlp.adam(rw, g[t - 1], rm, rv, lr, b1, b2, eps, t)
        # moments: a few roundings each; the step is lr * O(1), a few ulps of it
        np.testing.assert_allclose(_np(tm), rm, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(_np(tv), rv, rtol=1e-5, atol=1e-9)
        np.testing.assert_allclose(_np(tw), rw, rtol=0, atol=1e-6)

    # masked argmin: identical FP32 inputs, so identical decisions (first on ties)
    Pq = np.round(P * 4).astype(np.float32)   # many ties
    Mq = M.copy()
    Mq[5] = 0
    idx = spc.mlp_masked_argmin(torch.from_numpy(Pq).to(DEV), torch.from_numpy(Mq).to(DEV))
    np.testing.assert_array_equal(idx.cpu().numpy(), omlp.masked_argmin(Pq, Mq))
    for pref, margin in ((0, 0.0), (2, 0.25), (Pq.shape[1] - 1, 1.0)):
        idx = spc.mlp_masked_argmin(torch.from_numpy(Pq).to(DEV), torch.from_numpy(Mq).to(DEV),
                                    pref=pref, margin=margin)
        np.testing.assert_array_equal(idx.cpu().numpy(),
                                      omlp.masked_argmin(Pq, Mq, pref=pref, margin=margin))


# ------------------------------------------------------------- training

def test_training_matches_oracle_trajectory():
    """20 full-batch Adam steps of the device MLP against the FP64 oracle run
    from the same initial parameters."""
    from paper_2404_19638_amd.selector import MLP
    n = 300
    X = np.abs(_rand((n, 23), 81))
    T = _rand((n, 10), 82) + 1.0
    M = (synth.uniform_f32(83, n * 10).reshape(n, 10) > -0.4).astype(np.float32)
    net = MLP([23, 16, 16, 10], 5, DEV)
    layers = [(_np(W), _np(b)) for W, b in zip(net.W, net.b)]
    tX, tT, tM = (torch.from_numpy(a).to(DEV) for a in (X, T, M))
    lr = 3e-3
    # the device takes FP32 hyperparameters; the oracle uses the same rounded values
    flr, b1, b2, eps = (float(np.float32(x)) for x in (lr, 0.9, 0.999, 1e-8))
    mom = [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(b), np.zeros_like(b))
           for W, b in layers]
    losses_dev, losses_ref = [], []
    for t in range(1, 21):
        loss, grads = net.loss_and_grads(tX, tT, tM)
        rloss, rgrads = omlp.mlp_loss_grads(layers, X, T, M)
        if t == 1:
            for (gW, gb), (rW, rb) in zip(grads, rgrads):
                np.testing.assert_allclose(_np(gW), rW, rtol=1e-4, atol=1e-5 * np.abs(rW).max())
                np.testing.assert_allclose(_np(gb), rb, rtol=1e-4, atol=1e-5 * np.abs(rb).max())
        net.step(grads, lr)
        new = []
        for (W, b), (gW, gb), (mW, vW, mb, vb) in zip(layers, rgrads, mom):
            W, mW, vW = omlp.adam(W, gW, mW, vW, flr, b1, b2, eps, t)
            b, mb, vb = omlp.adam(b, gb, mb, vb, flr, b1, b2, eps, t)
            new.append(((W, b), (mW, vW, mb, vb)))
        layers = [x for x, _ in new]
        mom = [y for _, y in new]
        losses_dev.append(loss.item())
        losses_ref.append(rloss)
    _say("trajectory", [f"{a:.5f}/{b:.5f}" for a, b in zip(losses_dev[::5], losses_ref[::5])])
    np.testing.assert_allclose(losses_dev, losses_ref, rtol=1e-3)
    assert losses_ref[-1] < 0.7 * losses_ref[0]


# ------------------------------------------------------- selector end to end

def test_selector_small_end_to_end():
    """A reduced selector workload (32 blocks up to 2^14 rows, kz 16 and 64,
    FP32 and BF16): autotune, train on 24 blocks, judge on the other 8."""
    from paper_2404_19638_amd import selector as S
    blocks = [synth.selector_block(i, lg_hi=14, deg_hi=32) for i in range(32)]
    recs = S.collect(blocks, ks=(16, 64), reps=3, log=_say)
    train, held = synth.selector_split(32, 24)
    rtrain = [r for r in recs if r["block"] in set(train)]
    rheld = [r for r in recs if r["block"] in set(held)]
    sel = S.Selector((32, 32))
    for op in ("sddmm", "spmm", "sddmm_spmm"):
        X, T, M = S.dataset(rtrain, op)
        hist = sel.fit(op, X, T, M, steps=1500, log_every=500)
        assert hist[-1][1] < 0.5 * hist[0][1], hist
        fixed = S.best_fixed(rtrain, op)
        jt = S.judge(sel, rtrain, op, fixed)
        jh = S.judge(sel, rheld, op, fixed)
        _say(f"SELECTOR_SMALL {op}: train regret {jt['regret_geomean']:.4f} (default "
             f"{jt['default_regret_geomean']:.4f}); held-out regret {jh['regret_geomean']:.4f} "
             f"p90 {jh['regret_p90']:.4f} (default {jh['default_regret_geomean']:.4f}, fixed "
             f"{jh['fixed_regret_geomean']:.4f}); gain vs default {jh['gain_vs_default_geomean']:.4f}")
        # Fitted on the training blocks, the network is at least as good as the
        # library default and the best single variant there, up to 2% of timing
        # noise (the labels are timings of a few calls each); on the 8 held-out
        # blocks it stays within 15% of the exhaustive search (the full
        # 512-block evaluation is the selector workload run).
        best_fixed = min(jt["default_regret_geomean"], jt["fixed_regret_geomean"])
        assert jt["regret_geomean"] <= best_fixed + 0.02, jt
        assert jh["regret_geomean"] < 0.15 and jh["regret_max"] < 3.0, jh
        # it keeps the default unless it predicts a clear gain, so on the
        # held-out blocks it is no worse than the default beyond timing noise
        assert jh["regret_geomean"] <= jh["default_regret_geomean"] + 0.01, jh


def test_selector_gain_on_recorded_held_out_blocks():
    """The committed networks (trained on the GPU on the 384 training blocks of
    the selector workload, each with the keep-default margin chosen on those
    blocks) judged on the autotuner's recorded timings of the 128 held-out
    blocks (1024 instances per operation): no operation's held-out
    geometric-mean regret against the exhaustive autotuner is above the
    library default's, at least one is below it (the network gains over the
    method without it), and every one gains over the best single fixed
    variant.  Inference runs in the library's MLP and argmin kernels."""
    import os
    from paper_2404_19638_amd import selector as S
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sel = S.Selector.from_state(S.load_weights(os.path.join(root, "paper_2404_19638_amd",
                                                            "selector_weights.json")), DEV)
    recs = S.load_records_npz(os.path.join(root, "tests", "data",
                                           "selector_heldout_records.npz"))
    train, held = synth.selector_split(512, 384)
    assert {r["block"] for r in recs} <= set(held)
    gains = []
    for op in ("sddmm", "spmm", "sddmm_spmm"):
        assert sel.cands[op][0] == -1                      # the default is an output
        j = S.judge(sel, recs, op, S.best_fixed(recs, op))
        _say(f"SELECTOR_HELDOUT {op}: n {j['n']} margin {sel.margin_for(op):.4f} regret "
             f"{j['regret_geomean']:.4f} (default {j['default_regret_geomean']:.4f}, fixed "
             f"{j['fixed_regret_geomean']:.4f}); gain vs default {j['gain_vs_default_geomean']:.4f}")
        assert j["n"] == 1024
        assert j["regret_geomean"] <= j["default_regret_geomean"] + 1e-12, j
        assert j["gain_vs_fixed_geomean"] > 1.0, j
        gains.append(j["gain_vs_default_geomean"])
    assert max(gains) > 1.0, gains


def test_selector_choose_and_fallback():
    from paper_2404_19638_amd import selector as S
    spc = _spc()
    blocks = [synth.selector_block(i, lg_hi=13, deg_hi=16) for i in range(6)]
    recs = S.collect(blocks, ks=(16, 32), dtypes=(spc.F32,), ops=("sddmm",), reps=2)
    sel = S.Selector((16,))
    X, T, M = S.dataset(recs, "sddmm")
    sel.fit("sddmm", X, T, M, steps=200)
    b = blocks[2]
    plan = spc.plan_create_coo(torch.from_numpy(b["rows"]).to(DEV),
                               torch.from_numpy(b["cols"]).to(DEV), (0, b["n"]), (0, b["n"]))
    A = torch.rand((plan.R, 64), device=DEV)
    B = torch.rand((plan.C, 64), device=DEV)
    v, src = sel.choose(plan, "sddmm", 16, spc.F32)
    assert src == "mlp" and spc.variant_check(spc.OP_SDDMM, 16, spc.F32, v) == spc.OK
    out = spc.sddmm(plan, None, A[:, :16].contiguous(), B[:, :16].contiguous(), variant=v)
    ref = spc.sddmm(plan, None, A[:, :16].contiguous(), B[:, :16].contiguous())
    torch.testing.assert_close(out, ref, rtol=1e-5, atol=1e-5)
    # kz = 64 lies outside the kz range seen in training: the autotuner decides
    v2, src2 = sel.choose(plan, "sddmm", 64, spc.F32, A=A, B=B)
    assert src2 == "autotune" and spc.variant_check(spc.OP_SDDMM, 64, spc.F32, v2) == spc.OK
    # an operation without a model also falls back, and needs the operands
    with pytest.raises(ValueError):
        sel.choose(plan, "spmm", 16, spc.F32)
