"""Host-side logic of the variant selector (CPU only): training targets,
candidate masks, the best fixed variant, the weight file round trip and the
selector workload's generator and split."""
import math

import numpy as np

from paper_2404_19638_amd import selector as S
from paper_2404_19638_amd import spc3d as spc
from paper_2404_19638_amd import synth
from paper_2404_19638_amd import tune


def test_candidates_and_masks():
    sd, sp = tune.candidates("sddmm"), tune.candidates("spmm")
    assert len(sd) == len(set(sd)) and len(sp) == len(set(sp))
    assert all(not (v >> 8) & 3 for v in sd)          # SDDMM ignores the SpMM bits
    assert set(sd) < set(sp) and tune.candidates("sddmm_spmm") == sp
    # the network's outputs: the library default (-1) first, then every variant
    assert S.candidates("spmm") == [-1] + sp and S.candidates("sddmm") == [-1] + sd
    m = S.valid_mask("spmm", 32, spc.F32)
    assert m.shape == (len(sp) + 1,) and set(np.unique(m)) <= {0.0, 1.0} and m[0] == 1.0
    for v, ok in zip(S.candidates("spmm"), m):
        assert bool(ok) == (spc.variant_check(spc.OP_SPMM, 32, spc.F32, v) == spc.OK)
    # kz = 128 FP32 needs at least 8 lanes per entry
    m128 = S.valid_mask("sddmm", 128, spc.F32)
    assert all(not ok for v, ok in zip(S.candidates("sddmm"), m128) if v >= 0 and (v & 15) < 3)


def test_targets_are_capped_log_slowdowns():
    c = S.candidates("sddmm")
    assert c[0] == -1
    t = {c[1]: 1.0, c[2]: 2.0, c[3]: 100.0, -1: 1.5}
    T, M = S.targets(t, "sddmm")
    assert T[1] == 0.0 and T[2] == 1.0 and T[3] == S.TARGET_CAP
    assert T[0] == math.log2(1.5)
    assert M[:4].tolist() == [1, 1, 1, 1] and M[4:].sum() == 0 and T[4:].sum() == 0


def _rec(op, timings, block=0):
    return dict(op=op, block=block, kz=32, dtype=0, nnz=100, kind="uniform",
                features=np.zeros(S.NFEAT, np.float32), timings=timings)


def test_best_fixed_uses_the_operation_and_runnable_variants():
    a, b, c = tune.candidates("spmm")[:3]
    recs = [_rec("spmm", {a: 1.0, b: 2.0, c: 0.5, -1: 1.0}),
            _rec("spmm", {a: 1.0, b: 1.1, -1: 1.0}),                 # c cannot run here
            _rec("sddmm", {a: 9.0, b: 0.1, -1: 1.0})]                # another operation
    # c is fastest where it runs but does not run everywhere; b loses on spmm
    assert S.best_fixed(recs, "spmm") == a
    # when no candidate runs everywhere, a missing one counts as the default
    recs2 = [_rec("spmm", {a: 1.0, -1: 2.0}), _rec("spmm", {b: 1.0, -1: 4.0})]
    assert S.best_fixed(recs2, "spmm") == b


def test_weight_file_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    st = dict(hidden=[4], seed=3, cands={"spmm": [3, 19]},
              models={"spmm": dict(sizes=[S.NFEAT, 4, 2],
                                   W=[rng.standard_normal((4, S.NFEAT)).astype(np.float32).tolist(),
                                      rng.standard_normal((2, 4)).astype(np.float32).tolist()],
                                   b=[[0.5] * 4, [1.5, -2.0]])},
              lo={"spmm": [0.0] * S.NFEAT}, hi={"spmm": [1.0] * S.NFEAT},
              margins={"spmm": 0.0, "sddmm": None})
    p = tmp_path / "w.json"
    S.save_weights(st, str(p), note="test")
    back = S.load_weights(str(p))
    assert back["cands"] == st["cands"] and back["hidden"] == [4]
    assert back["margins"] == {"spmm": 0.0, "sddmm": None}   # None: always the default
    for x, y in zip(back["models"]["spmm"]["W"], st["models"]["spmm"]["W"]):
        np.testing.assert_array_equal(np.float32(x), np.float32(y))
    assert back["models"]["spmm"]["b"][1] == [1.5, -2.0]


def test_selector_workload_generator_and_split():
    tr, ho = synth.selector_split()
    assert len(tr) == 384 and len(ho) == 128 and not set(tr) & set(ho)
    assert sorted(tr + ho) == list(range(512))
    assert synth.selector_split() == (tr, ho)                 # seeded
    for i in (0, 1, 7):
        b = synth.selector_block(i, lg_hi=14)
        n = b["n"]
        assert 2 ** 10 - 1 <= n <= 2 ** 14 + 1 and 4 <= b["deg"] <= 64
        assert b["kind"] == ("uniform" if i % 2 == 0 else "rmat")
        assert b["rows"].min() >= 0 and b["rows"].max() < n and b["cols"].max() < n
        key = b["rows"] * n + b["cols"]
        assert np.unique(key).size == key.size                # distinct entries
        if b["kind"] == "uniform":
            assert key.size == min(int(round(b["deg"] * n)), n * n // 2)
        again = synth.selector_block(i, lg_hi=14)
        np.testing.assert_array_equal(again["rows"], b["rows"])
    # sizes over the full workload are log-uniform: both ends are reached and
    # about half the blocks lie below the geometric middle 2^14
    lg = [10 + 8 * synth._unit(synth.SELECTOR_SEED, 4 * i) for i in range(512)]
    assert min(lg) < 10.1 and max(lg) > 17.9
    assert 0.4 < np.mean(np.array(lg) < 14) < 0.6
    assert math.isclose(S.TARGET_CAP, 3.0)


def test_margins_survive_the_state_round_trip():
    import math
    sel = S.Selector((4,), device="cpu")
    sel.margins = {"spmm": 0.0, "sddmm": math.inf}
    st = sel.state()
    assert st["margins"] == {"spmm": 0.0, "sddmm": None}
    back = S.Selector.from_state(st, device="cpu")
    assert back.margin_for("spmm") == 0.0 and math.isinf(back.margin_for("sddmm"))
    assert back.margin_for("sddmm_spmm") == S.KEEP_DEFAULT_MARGIN   # not chosen: the constant
