"""Pins of the oracle's owner-grouped localization (Method 2, SpC-SB / SpC-RB:
local ids ordered by (group key, global id)), host only."""
import numpy as np
import pytest

import oracle


def _case(seed, nr=50, nc=60, nnz=300, lo_r=1000, lo_c=7):
    rng = np.random.default_rng(seed)
    cells = rng.choice(nr * nc, size=nnz, replace=False)
    rows = (cells // nc + lo_r).astype(np.int64)
    cols = (cells % nc + lo_c).astype(np.int64)
    return rows, cols, (lo_r, lo_r + nr), (lo_c, lo_c + nc)


@pytest.mark.parametrize("seed,ng_r,ng_c", [(1, 3, 5), (2, 1, 7), (3, 64, 2)])
def test_grouped_relabel_brute_force(seed, ng_r, ng_c):
    rows, cols, rr, cr = _case(seed)
    rng = np.random.default_rng(seed + 100)
    gr = rng.integers(0, ng_r, rr[1] - rr[0]).astype(np.int32)
    gc = rng.integers(0, ng_c, cr[1] - cr[0]).astype(np.int32)
    ref = oracle.relabel(rows, cols, rr, cr, csc=True, group_r=gr, ngroups_r=ng_r, group_c=gc,
                         ngroups_c=ng_c)
    # local ids: the used ids sorted by (group, id), by brute force
    for gid, lo, g, key in ((rows, rr[0], gr, "r"), (cols, cr[0], gc, "c")):
        used = sorted(set(int(v) for v in gid), key=lambda v: (int(g[v - lo]), v))
        assert ref[f"gmap_{key}"].tolist() == used
        lmap = ref[f"lmap_{key}"]
        for j, v in enumerate(used):
            assert lmap[v - lo] == j
        assert (lmap >= 0).sum() == len(used)
    # every slot maps back to its caller entry; rows sorted by (local col, caller)
    rp, ci, perm = ref["rowptr"], ref["colidx"], ref["perm"]
    lr = np.repeat(np.arange(ref["R"]), np.diff(rp))
    assert np.array_equal(ref["gmap_r"][lr], rows[perm])
    assert np.array_equal(ref["gmap_c"][ci], cols[perm])
    key = lr.astype(np.int64) * ref["C"] + ci
    assert np.all(np.diff(key) > 0)
    # column-major view consistent with the row-major one
    cp, ri, st = ref["colptr"], ref["rowidx_t"], ref["slot_t"]
    lc = np.repeat(np.arange(ref["C"]), np.diff(cp))
    assert np.array_equal(ci[st], lc) and np.array_equal(lr[st], ri)


def test_single_group_is_the_plain_order_and_bad_keys_raise():
    rows, cols, rr, cr = _case(5)
    plain = oracle.relabel(rows, cols, rr, cr)
    zero = oracle.relabel(rows, cols, rr, cr, group_r=np.zeros(rr[1] - rr[0], np.int32),
                          ngroups_r=1, group_c=np.zeros(cr[1] - cr[0], np.int32), ngroups_c=1)
    for k in ("gmap_r", "gmap_c", "lmap_r", "lmap_c", "rowptr", "colidx", "perm"):
        assert np.array_equal(plain[k], zero[k]), k
    bad = np.zeros(rr[1] - rr[0], np.int32)
    bad[rows[0] - rr[0]] = 3
    with pytest.raises(ValueError):
        oracle.relabel(rows, cols, rr, cr, group_r=bad, ngroups_r=3)
    # a bad key on an id the block does not use is ignored
    unused = sorted(set(range(rr[0], rr[1])) - set(rows.tolist()))
    if unused:
        ok = np.zeros(rr[1] - rr[0], np.int32)
        ok[unused[0] - rr[0]] = 99
        oracle.relabel(rows, cols, rr, cr, group_r=ok, ngroups_r=1)
