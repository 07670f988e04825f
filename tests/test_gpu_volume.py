"""Dist3D communication accounting on the GPU (relabel per block, lambda and
Algorithm 1 owners in spc3d_lambda_owners) against the oracle's relabel and
brute-force owner choice: every integer result bit-exact, on square and
non-square grids of R-MAT patterns; and the out-of-range error path."""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth
from test_volume_host import _oracle_dist3d

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("scale,X,Y,Z", [(12, 4, 4, 1), (13, 6, 5, 2), (14, 8, 8, 4)])
def test_owner_kernel_and_simulator_match_oracle(scale, X, Y, Z):
    from paper_2404_19638_amd import spc3d as spc
    from paper_2404_19638_amd.volume import bounds, simulate
    n = 1 << scale
    rows, cols = synth.rmat_block(scale, 16 << scale, 500 + scale, (0, n), (0, n))
    rnd_r = synth.draws_u64(600 + scale, n)
    rnd_c = synth.draws_u64(700 + scale, n)
    _say(f"volume scale={scale} grid={X}x{Y}x{Z} nnz={rows.size}")
    want, orr, occ, (rb, cb, bx, by) = _oracle_dist3d(rows, cols, n, n, X, Y, Z, rnd_r, rnd_c)
    # the owner kernel alone, on the plans' globalMaps of block row 1
    x = 1
    gm = []
    for y in range(Y):
        s = (bx == x) & (by == y)
        plan = spc.plan_create_coo(torch.from_numpy(rows[s]).to(DEV),
                                   torch.from_numpy(cols[s]).to(DEV),
                                   (int(rb[x]), int(rb[x + 1])), (int(cb[y]), int(cb[y + 1])))
        gm.append((plan, plan.maps()["gmap_r"]))
    lo, hi = int(rb[x]), int(rb[x + 1])
    rr = torch.from_numpy(rnd_r[lo:hi].view(np.int64)).to(DEV)
    got = spc.lambda_owners([g for _, g in gm], lo, hi, rr)
    for k in ("lambda_", "owner", "owned", "comm"):
        np.testing.assert_array_equal(got[k].cpu().numpy(), orr[x][k], err_msg=k)
    # without draws: the lowest candidate
    got0 = spc.lambda_owners([g for _, g in gm], lo, hi, None)
    ref0 = oracle.lambda_owners([g.cpu().numpy() for _, g in gm], lo, hi)
    np.testing.assert_array_equal(got0["owner"].cpu().numpy(), ref0["owner"])
    # the whole simulator
    rep = simulate(rows, cols, n, n, X, Y, Z, rnd_r, rnd_c, device=DEV)
    for k, v in want.items():
        assert rep[k] == v, (k, rep[k], v)


def test_ids_outside_the_range_are_reported():
    from paper_2404_19638_amd import spc3d as spc
    g = [torch.tensor([3, 5, 9], dtype=torch.int64, device=DEV),
         torch.tensor([4, 12], dtype=torch.int64, device=DEV)]
    with pytest.raises(spc.Spc3dError) as ei:
        spc.lambda_owners(g, 0, 10)
    assert ei.value.status == spc.ERR_OUT_OF_RANGE
    ok = spc.lambda_owners(g[:1], 0, 10)
    assert ok["lambda_"].cpu().numpy().tolist() == [0, 0, 0, 1, 0, 1, 0, 0, 0, 1]


def test_full_size_grid_matches_oracle_and_times_both():
    """R-MAT 2^20, average degree 32 on the 10 x 10 x 9 grid (P = 900): every
    count of the GPU simulator equals the oracle's accounting; both timed."""
    import json
    import time
    from paper_2404_19638_amd.volume import simulate
    scale, X, Y, Z = 20, 10, 10, 9
    n = 1 << scale
    rows, cols = synth.rmat_block(scale, 32 << scale, 2409, (0, n), (0, n))
    rnd_r = synth.draws_u64(2410, n)
    rnd_c = synth.draws_u64(2411, n)
    _say(f"volume full size nnz={rows.size}")
    simulate(rows[:1000], cols[:1000], n, n, 2, 2, 1, rnd_r, rnd_c, device=DEV)   # warm-up
    t0 = time.perf_counter()
    rep = simulate(rows, cols, n, n, X, Y, Z, rnd_r, rnd_c, device=DEV)
    t_gpu = time.perf_counter() - t0
    t0 = time.perf_counter()
    want, _, _, _ = _oracle_dist3d(rows, cols, n, n, X, Y, Z, rnd_r, rnd_c)
    t_cpu = time.perf_counter() - t0
    for k, v in want.items():
        assert rep[k] == v, (k, rep[k], v)
    print("VOLUME_REPORT " + json.dumps({
        "workload": "rmat20-deg32", "grid": [X, Y, Z], "max_recv_per_K": rep["max_recv_per_K"],
        "dense3d_recv_per_K": rep["dense3d_recv_per_K"], "improvement": rep["improvement"],
        "simulator_s": round(t_gpu, 3), "oracle_s": round(t_cpu, 3)}), flush=True)
