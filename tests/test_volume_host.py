"""Pins of the lambda / Algorithm 1 oracle and of the Dist3D volume accounting
(host logic, no GPU).

- lambda and the receive sets against brute force from the raw COO of tiny
  patterns (Python sets of the parts each row / column occurs in);
- owners are always candidates, the draws pick the candidate of the stated
  rank, owned counts add up;
- the paper's total-volume identity: the processors receive
  sum_i (lambda_i - 1) + sum_j (lambda_j - 1) rows in all;
- a dense pattern with owners spread evenly reproduces the Dense3D receive
  volume (A_size + B_size)(sqrt(P/Z) - 1)/P exactly.
"""
import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth
from paper_2404_19638_amd.volume import account, bounds


def _blocks(rows, cols, M, N, X, Y):
    rb, cb = bounds(M, X), bounds(N, Y)
    bx = np.searchsorted(rb, rows, side="right") - 1
    by = np.searchsorted(cb, cols, side="right") - 1
    return rb, cb, bx, by


def _oracle_dist3d(rows, cols, M, N, X, Y, Z, rnd_r, rnd_c):
    """Accounting from the oracle's relabel and owner choice."""
    rb, cb, bx, by = _blocks(rows, cols, M, N, X, Y)
    R = np.zeros((X, Y), np.int64)
    C = np.zeros((X, Y), np.int64)
    nnz = np.zeros((X, Y), np.int64)
    gr = [[np.zeros(0, np.int64)] * Y for _ in range(X)]
    gc = [[np.zeros(0, np.int64)] * Y for _ in range(X)]
    for x in range(X):
        for y in range(Y):
            s = (bx == x) & (by == y)
            if not s.any():
                continue
            ref = oracle.relabel(rows[s], cols[s], (rb[x], rb[x + 1]), (cb[y], cb[y + 1]))
            R[x, y], C[x, y], nnz[x, y] = ref["R"], ref["C"], s.sum()
            gr[x][y], gc[x][y] = ref["gmap_r"], ref["gmap_c"]
    orr = [oracle.lambda_owners(gr[x], rb[x], rb[x + 1], rnd_r[rb[x]:rb[x + 1]]) for x in range(X)]
    occ = [oracle.lambda_owners([gc[x][y] for x in range(X)], cb[y], cb[y + 1],
                                rnd_c[cb[y]:cb[y + 1]]) for y in range(Y)]
    rep = account(M, N, X, Y, Z, R, C, np.stack([o["owned"] for o in orr]),
                  np.stack([o["owned"] for o in occ]), [o["comm"] for o in orr],
                  [o["comm"] for o in occ], nnz)
    return rep, orr, occ, (rb, cb, bx, by)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lambda_and_receive_sets_brute_force(seed):
    rng = np.random.default_rng(seed)
    M, N, X, Y, Z = 37, 41, 3, 4, 2
    nnz = 150
    cells = rng.choice(M * N, size=nnz, replace=False)
    rows, cols = (cells // N).astype(np.int64), (cells % N).astype(np.int64)
    rnd_r = synth.draws_u64(seed + 10, M)
    rnd_c = synth.draws_u64(seed + 20, N)
    rep, orr, occ, (rb, cb, bx, by) = _oracle_dist3d(rows, cols, M, N, X, Y, Z, rnd_r, rnd_c)
    # brute force: which column blocks each row occurs in, which row blocks each column
    row_parts = {i: set() for i in range(M)}
    col_parts = {j: set() for j in range(N)}
    for i, j, x, y in zip(rows, cols, bx, by):
        row_parts[int(i)].add(int(y))
        col_parts[int(j)].add(int(x))
    recv = np.zeros((X, Y), np.int64)
    for x in range(X):
        lam, own = orr[x]["lambda_"], orr[x]["owner"]
        for i in range(rb[x], rb[x + 1]):
            parts = row_parts[i]
            assert lam[i - rb[x]] == len(parts)
            if parts:
                o = int(own[i - rb[x]])
                assert o in parts
                # the draw picks the candidate of rank floor(r * lambda / 2^64)
                k = (int(rnd_r[i]) * len(parts)) >> 64
                assert o == sorted(parts)[k]
                for y in parts - {o}:
                    recv[x, y] += 1
            else:
                assert own[i - rb[x]] == -1
    for y in range(Y):
        lam, own = occ[y]["lambda_"], occ[y]["owner"]
        for j in range(cb[y], cb[y + 1]):
            parts = col_parts[j]
            assert lam[j - cb[y]] == len(parts)
            if parts:
                o = int(own[j - cb[y]])
                assert o in parts and o == sorted(parts)[(int(rnd_c[j]) * len(parts)) >> 64]
                for x in parts - {o}:
                    recv[x, y] += 1
    assert rep["max_recv_per_K"] == recv.max() / Z
    # identity: total received rows = sum (lambda - 1) over used rows and columns
    total = sum(len(p) - 1 for p in row_parts.values() if p) + \
        sum(len(p) - 1 for p in col_parts.values() if p)
    assert rep["identity_rows"] == total == recv.sum()
    # every received row is sent once by its owner; buffers only add memory
    assert rep["total_send_rows"] == total
    assert rep["max_mem_nb_per_K"] <= rep["max_mem_rb_per_K"] <= rep["max_mem_bb_per_K"]
    # owned counts add up to the used ids; comm rows sum to the receive sets
    for x in range(X):
        assert orr[x]["owned"].sum() == sum(1 for i in range(rb[x], rb[x + 1]) if row_parts[i])
        assert np.all(np.diag(orr[x]["comm"]) == 0)


def test_dense_pattern_reproduces_dense3d_formula():
    """All cells stored, owners spread round-robin by the draws: each processor
    receives exactly (M/X)(Y-1)/Y + (N/Y)(X-1)/X rows, the Dense3D volume."""
    M = N = 144   # block ranges divisible by the parts: owners split exactly evenly
    for X, Z in ((4, 1), (3, 2), (2, 4)):
        Y = X
        cells = np.arange(M * N, dtype=np.int64)
        rows, cols = cells // N, cells % N
        # draw of id i selects rank (i mod parts) among the parts (all of them)
        rnd_r = np.array([((i % Y) * 2 ** 64 + 2 ** 63) // Y for i in range(M)], np.uint64)
        rnd_c = np.array([((j % X) * 2 ** 64 + 2 ** 63) // X for j in range(N)], np.uint64)
        rep, orr, _, _ = _oracle_dist3d(rows, cols, M, N, X, Y, Z, rnd_r, rnd_c)
        assert all(np.all(o["lambda_"] == Y) for o in orr)
        P = X * Y * Z
        want = (M + N) * (np.sqrt(P / Z) - 1) / P
        assert rep["dense3d_formula_per_K"] == pytest.approx(want)
        assert rep["max_recv_per_K"] == pytest.approx(want)
        assert rep["mean_recv_per_K"] == pytest.approx(want)
        assert rep["max_mem_per_K"] == pytest.approx(rep["dense3d_mem_per_K"])


def test_no_draws_pick_the_lowest_candidate():
    g = [np.array([0, 2, 3]), np.array([2, 3, 4]), np.array([3])]
    r = oracle.lambda_owners(g, 0, 6)
    assert r["lambda_"].tolist() == [1, 0, 2, 3, 1, 0]
    assert r["owner"].tolist() == [0, -1, 0, 0, 1, -1]
    assert r["owned"].tolist() == [3, 1, 0]
    assert r["comm"].tolist() == [[0, 0, 0], [2, 0, 0], [1, 0, 0]]


def test_grid_2d_near_square():
    from paper_2404_19638_amd.volume import grid_2d
    assert [grid_2d(900, z) for z in (1, 2, 4, 9)] == [(30, 30), (18, 25), (15, 15), (10, 10)]
    assert grid_2d(7, 1) == (1, 7)
    with pytest.raises(ValueError):
        grid_2d(900, 7)


def test_dense_pattern_non_square_grid():
    """X != Y (the paper's Z = 2 at P = 900 needs one): with every cell stored
    and owners spread evenly, every processor receives exactly
    (M/X)(Y-1)/Y + (N/Y)(X-1)/X rows per slice, the Dense3D volume."""
    M, N = 120, 240   # block ranges divisible by the parts: owners split exactly evenly
    for X, Y, Z in ((2, 3, 1), (3, 5, 2), (4, 6, 1)):
        cells = np.arange(M * N, dtype=np.int64)
        rows, cols = cells // N, cells % N
        rnd_r = np.array([((i % Y) * 2 ** 64 + 2 ** 63) // Y for i in range(M)], np.uint64)
        rnd_c = np.array([((j % X) * 2 ** 64 + 2 ** 63) // X for j in range(N)], np.uint64)
        rep, _, _, _ = _oracle_dist3d(rows, cols, M, N, X, Y, Z, rnd_r, rnd_c)
        want = ((M / X) * (Y - 1) / Y + (N / Y) * (X - 1) / X) / Z
        assert rep["dense3d_recv_per_K"] == pytest.approx(want)
        assert rep["max_recv_per_K"] == pytest.approx(want)
        assert rep["mean_recv_per_K"] == pytest.approx(want)
        assert rep["dense3d_formula_per_K"] is None
