"""Communication accounting of a Dist3D distribution on one GPU.

The paper measures sparsity-aware communication by the volume each processor
receives (Section "Sparsity-aware Communication Analysis of 3D SDDMM"): on an
X x Y x Z grid, processor P_{x,y,z} holds block S_{x,y} (rows in the x-th of X
equal row ranges, columns in the y-th of Y column ranges) and the z-th K/Z
slice of the dense rows it uses.  Row i of A is used by the lambda_i
processors of its row group whose block has a nonzero in row i; Algorithm 1
("Parallel lambda-aware random distribution") makes one of them its owner,
and every other user receives it in the PreComm phase.  With I_a and J_a the
rows and columns of S_{x,y} that P_a uses but does not own, P_a receives
(K/Z)(|I_a| + |J_a|) words; Table 2 reports the maximum over processors,
divided by K.  Dense3D (Section "Sparsity-agnostic parallel algorithms", 3D
paragraph) receives the whole row and column blocks:
(M/X)(Y-1)/Y + (N/Y)(X-1)/X rows per K/Z columns, i.e. (A_size + B_size)
(sqrt(P/Z) - 1)/P words when X = Y.

This module localizes every block with the library's relabel (one plan per
block, its globalMap gives the rows and columns the block uses), runs
Algorithm 1 per block row and block column with spc3d_lambda_owners, and
accounts the volumes, message counts and memory of both schemes.  The owner
of a row is the same for the Z slices (the candidates do not depend on z).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

from . import spc3d as spc


def grid_2d(P: int, Z: int) -> tuple:
    """X <= Y with X * Y = P / Z and X as close to sqrt(P / Z) as the divisors
    allow (X = Y when P / Z is a square)."""
    if P % Z:
        raise ValueError(f"Z={Z} does not divide P={P}")
    q = P // Z
    X = max(d for d in range(1, int(q ** 0.5) + 1) if q % d == 0)
    return X, q // X


def bounds(n: int, parts: int) -> np.ndarray:
    """Equal contiguous ranges: part p covers [b[p], b[p+1])."""
    return np.array([p * n // parts for p in range(parts + 1)], dtype=np.int64)


def account(M, N, X, Y, Z, R, C, owned_r, owned_c, comm_r, comm_c, nnz_blk) -> dict:
    """Volumes from the per-block counts (host arithmetic only).

    R, C, nnz_blk: [X, Y] rows, columns and nonzeros of each block;
    owned_r[x, y]: rows of block row x owned by part y; owned_c[y, x]: columns
    of block column y owned by part x; comm_r[x][y, q]: rows part y of block
    row x receives from part q; comm_c[y][x, q] likewise for columns.
    Volumes are in rows (words / (K/Z)); "per_K" values are words / K."""
    R = np.asarray(R, np.int64)
    C = np.asarray(C, np.int64)
    I = R - np.asarray(owned_r, np.int64)                    # [X, Y]
    J = C - np.asarray(owned_c, np.int64).T                  # [X, Y]
    recv_rows = I + J
    msgs = np.zeros((X, Y), np.int64)
    post_rows = np.zeros((X, Y), np.int64)   # SpMM PostComm: partial rows arriving at owners
    send_rows = np.zeros((X, Y), np.int64)   # PreComm: owned rows sent to the other users
    for x in range(X):
        msgs[x] += (np.asarray(comm_r[x]) > 0).sum(1)
        post_rows[x] += np.asarray(comm_r[x]).sum(0)
        send_rows[x] += np.asarray(comm_r[x]).sum(0)
    for y in range(Y):
        msgs[:, y] += (np.asarray(comm_c[y]) > 0).sum(1)
        send_rows[:, y] += np.asarray(comm_c[y]).sum(0)
    # dense-row memory of the three transports of Section "Sparse communication
    # model" (rows of K/Z columns): SpC-NB keeps only the rows the block uses;
    # SpC-RB receives in place but packs what it sends; SpC-BB packs both ways
    used = R + C
    mem_nb, mem_rb, mem_bb = used, used + send_rows, used + send_rows + recv_rows
    dense_rows = (M / X) * (Y - 1) / Y + (N / Y) * (X - 1) / X
    P = X * Y * Z
    return dict(
        grid=[X, Y, Z], P=P,
        max_recv_per_K=float(recv_rows.max()) / Z,
        mean_recv_per_K=float(recv_rows.mean()) / Z,
        total_recv_per_K=float(recv_rows.sum()),            # summed over all P processors
        identity_rows=int(recv_rows.sum()),                  # = sum (lambda - 1) over rows and cols
        dense3d_recv_per_K=dense_rows / Z,
        dense3d_formula_per_K=(M + N) * (np.sqrt(P / Z) - 1) / P if X == Y else None,
        improvement=(dense_rows / Z) / max(float(recv_rows.max()) / Z, 1e-300),
        max_msgs=int(msgs.max()), mean_msgs=float(msgs.mean()),
        dense3d_msgs=(Y - 1) + (X - 1),
        max_spmm_postcomm_per_K=float(post_rows.max()) / Z,
        max_sddmm_reduce_scatter_words=float(np.asarray(nnz_blk).max()) * (Z - 1) / Z,
        max_mem_per_K=float((R + C).max()) / Z,
        dense3d_mem_per_K=(M / X + N / Y) / Z,
        total_send_rows=int(send_rows.sum()),              # = identity_rows
        max_send_per_K=float(send_rows.max()) / Z,
        max_mem_nb_per_K=float(mem_nb.max()) / Z,
        max_mem_rb_per_K=float(mem_rb.max()) / Z,
        max_mem_bb_per_K=float(mem_bb.max()) / Z,
    )


def simulate(rows, cols, M, N, X, Y, Z, rand_rows, rand_cols, device="cuda:0") -> dict:
    """Dist3D accounting of the global pattern (rows, cols) (int64 global ids,
    distinct entries) on an X x Y x Z grid.  rand_rows / rand_cols: M and N
    64-bit draws, one per row / column id, for Algorithm 1's random picks."""
    if X > 64 or Y > 64:
        raise ValueError("at most 64 parts per block row / column")
    t0 = time.perf_counter()
    rb, cb = bounds(M, X), bounds(N, Y)
    bx = np.searchsorted(rb, rows, side="right") - 1
    by = np.searchsorted(cb, cols, side="right") - 1
    key = bx * Y + by
    order = np.argsort(key, kind="stable")
    cnt = np.bincount(key, minlength=X * Y)
    off = np.concatenate([[0], np.cumsum(cnt)])
    R = np.zeros((X, Y), np.int64)
    C = np.zeros((X, Y), np.int64)
    gr = [[None] * Y for _ in range(X)]
    gc = [[None] * Y for _ in range(X)]
    plans = []
    for x in range(X):
        for y in range(Y):
            sel = order[off[x * Y + y]:off[x * Y + y + 1]]
            if sel.size == 0:
                continue
            plan = spc.plan_create_coo(torch.from_numpy(rows[sel]).to(device),
                                       torch.from_numpy(cols[sel]).to(device),
                                       (int(rb[x]), int(rb[x + 1])), (int(cb[y]), int(cb[y + 1])))
            m = plan.maps()
            R[x, y], C[x, y] = plan.R, plan.C
            gr[x][y], gc[x][y] = m["gmap_r"], m["gmap_c"]
            plans.append(plan)
    t_relabel = time.perf_counter() - t0
    rr = torch.from_numpy(rand_rows.view(np.int64)).to(device)
    rc = torch.from_numpy(rand_cols.view(np.int64)).to(device)
    owned_r = np.zeros((X, Y), np.int64)
    owned_c = np.zeros((Y, X), np.int64)
    comm_r, comm_c = [], []
    lam_hist = np.zeros(max(X, Y) + 1, np.int64)
    for x in range(X):
        lo, hi = int(rb[x]), int(rb[x + 1])
        o = spc.lambda_owners(gr[x], lo, hi, rr[lo:hi], device=device)
        owned_r[x] = o["owned"].cpu().numpy()
        comm_r.append(o["comm"].cpu().numpy())
        lam_hist += np.bincount(o["lambda_"].cpu().numpy(), minlength=lam_hist.size)[:lam_hist.size]
    for y in range(Y):
        lo, hi = int(cb[y]), int(cb[y + 1])
        o = spc.lambda_owners([gc[x][y] for x in range(X)], lo, hi, rc[lo:hi], device=device)
        owned_c[y] = o["owned"].cpu().numpy()
        comm_c.append(o["comm"].cpu().numpy())
    torch.cuda.synchronize()
    out = account(M, N, X, Y, Z, R, C, owned_r, owned_c, comm_r, comm_c, cnt.reshape(X, Y))
    out.update(nnz=int(rows.size), M=M, N=N, row_lambda_hist=lam_hist.tolist(),
               seconds_relabel=round(t_relabel, 3),
               seconds_total=round(time.perf_counter() - t0, 3))
    del plans
    return out


def main(argv=None):
    from . import synth
    ap = argparse.ArgumentParser(description="Dist3D receive volume of a synthetic R-MAT graph")
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--deg", type=int, default=32)
    ap.add_argument("--P", type=int, default=900)
    ap.add_argument("--Z", default="1,2,4,9")
    ap.add_argument("--seed", type=int, default=2409)
    a = ap.parse_args(argv)
    n = 1 << a.scale
    rows, cols = synth.rmat_block(a.scale, a.deg << a.scale, a.seed, (0, n), (0, n))
    rnd_r = synth.draws_u64(a.seed + 1, n)
    rnd_c = synth.draws_u64(a.seed + 2, n)
    for z in (int(v) for v in a.Z.split(",")):
        X, Y = grid_2d(a.P, z)
        rep = simulate(rows, cols, n, n, X, Y, z, rnd_r, rnd_c)
        rep["workload"] = f"rmat{a.scale}-deg{a.deg}"
        print("VOLUME " + json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
