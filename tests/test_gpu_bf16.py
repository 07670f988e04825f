"""BF16 inputs with FP32 accumulation (the precision extension) against the
FP64 oracle, with two references:

  (i)  the oracle on the BF16-rounded inputs isolates the GPU's accumulation,
       which must meet the FP32 bar |x - x*| <= 1e-5 M;
  (ii) the oracle on the original FP32 inputs gives the end-to-end error a
       user sees: each product a*b carries the two roundings to bfloat16
       (unit roundoff 2^-8 each), so |x - x*| <= (2^-7 + 2^-16 + 1e-5) M.

The full-size case is the precision workload (R-MAT 2^22 vertices, average
degree 32, K = 128) checked on sampled outputs; its error statistics are
printed as one JSON line.
"""
import json
import sys

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth
from helpers import assert_within_mag, error_report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"
E2E = 2.0 ** -7 + 2.0 ** -16 + 1e-5


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _np(t):
    return t.detach().cpu().numpy()


def _bf16_round(x):
    return oracle.bf16_to_f32(oracle.bf16_rne(x))


@pytest.mark.parametrize("kz", [32, 16, 64, 8])
def test_bf16_paths_against_both_references(kz):
    spc = _spc()
    p = synth.small_rmat(12, 8, 64, 41, row_range=(1 << 11, 1 << 12), col_range=(0, 1 << 11))
    k0 = 64 - kz
    _say(f"bf16 kz={kz} nnz={p.nnz}")
    ref = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range, csc=True)
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range, spc.BUILD_CSC)
    A = spc.gather(plan, spc.ROWS, torch.from_numpy(p.A_src).to(DEV), k0, kz, torch.bfloat16)
    B = spc.gather(plan, spc.COLS, torch.from_numpy(p.B_src).to(DEV), k0, kz, torch.bfloat16)
    vals = torch.from_numpy(p.vals[ref["perm"]]).to(DEV)
    Ar, Br = _bf16_round(p.A_src), _bf16_round(p.B_src)
    for v in (-1, spc.variant(3, 0), spc.variant(2, 3), spc.variant(4, 2)):
        out = spc.sddmm(plan, vals, A, B, kz, variant=v)
        Y = spc.spmm(plan, vals, B, 0, kz, variant=v)
        YT = spc.spmm(plan, vals, A, 1, kz, variant=v)
        fo, fy = spc.sddmm_spmm(plan, vals, A, B, kz, variant=v)
        for (Asrc, Bsrc, rel, tag) in ((Ar, Br, 1e-5, "rounded"), (p.A_src, p.B_src, E2E, "fp32")):
            o, m = oracle.sddmm(p.rows, p.cols, p.row_range[0], p.col_range[0], p.vals, Asrc, Bsrc,
                                k0, kz)
            assert_within_mag(_np(out), o[ref["perm"]], m[ref["perm"]], rel, f"sddmm {tag} v={v}")
            assert_within_mag(_np(fo), o[ref["perm"]], m[ref["perm"]], rel, f"fused sd {tag}")
            y, my = oracle.spmm(p.rows, p.cols, p.row_range[0], p.col_range[0], ref["lmap_r"],
                                ref["R"], p.vals, Bsrc, k0, kz)
            assert_within_mag(_np(Y), y, my, rel, f"spmm {tag} v={v}")
            assert_within_mag(_np(fy), y, my, rel, f"fused sp {tag}")
            yt, myt = oracle.spmm(p.cols, p.rows, p.col_range[0], p.row_range[0], ref["lmap_c"],
                                  ref["C"], p.vals, Asrc, k0, kz)
            assert_within_mag(_np(YT), yt, myt, rel, f"spmm^T {tag} v={v}")


def _sample_rows_oracle(p, rng, ns, Bsrc, k0, kz, lo_c, longest=64):
    """Oracle SpMM rows for ns sampled global rows plus the `longest` rows
    with the most entries (compact local ids)."""
    rows_g, counts = np.unique(p.rows, return_counts=True)
    top = rows_g[np.argsort(counts, kind="stable")[-longest:]]
    pick = np.union1d(rng.choice(rows_g, size=min(ns, rows_g.size), replace=False), top)
    sel = np.isin(p.rows, pick)
    rr = p.row_range
    lmap = np.full(rr[1] - rr[0], -1, np.int32)
    lmap[pick - rr[0]] = np.arange(pick.size, dtype=np.int32)
    y, m = oracle.spmm(p.rows[sel], p.cols[sel], rr[0], lo_c, lmap, pick.size, p.vals[sel], Bsrc,
                       k0, kz)
    return pick, y, m


def test_precision_workload_full_size():
    """R-MAT 2^22, degree 32, K=128 as one block: relabel invariants at full size,
    FP32 and BF16 SDDMM / SpMM on sampled outputs against the FP64 oracle (the
    SpMM sample holds 2,000 random rows and the 64 longest, up to 163K entries)."""
    spc = _spc()
    p = synth.precision()
    K = p.K
    _say(f"precision workload nnz={p.nnz}")
    rows = torch.from_numpy(p.rows).to(DEV)
    cols = torch.from_numpy(p.cols).to(DEV)
    plan = spc.plan_create_coo(rows, cols, p.row_range, p.col_range)
    m = plan.maps()
    # relabel: properties that fix the result uniquely, checked at full size
    gr = m["gmap_r"]
    assert plan.R == int(torch.unique(rows).numel())
    assert bool((gr[1:] > gr[:-1]).all())
    rp = m["rowptr"].long()
    assert int(rp[-1]) == p.nnz and bool((rp[1:] > rp[:-1]).all())
    perm = m["perm"].long()
    assert bool((torch.sort(perm)[0] == torch.arange(p.nnz, device=DEV)).all())
    lr = torch.repeat_interleave(torch.arange(plan.R, device=DEV), rp[1:] - rp[:-1])
    col_l = m["colidx"].long()
    assert bool((gr[lr] == rows[perm]).all()) and bool((m["gmap_c"][col_l] == cols[perm]).all())
    key = lr * plan.C + col_l
    assert bool((key[1:] > key[:-1]).all())          # distinct entries, sorted by (row, col)
    del lr, key, col_l, rows, cols
    vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, torch.from_numpy(p.vals).to(DEV))
    Asrc = torch.from_numpy(p.A_src).to(DEV)
    Bsrc = torch.from_numpy(p.B_src).to(DEV)
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(p.nnz, size=200_000, replace=False))
    perm_np = _np(perm)
    report = {"workload": "rmat22-deg32-whole-K128", "nnz": p.nnz, "R": plan.R, "C": plan.C}
    Ar, Br = _bf16_round(p.A_src), _bf16_round(p.B_src)
    for dt in (torch.float32, torch.bfloat16):
        name = "f32" if dt == torch.float32 else "bf16"
        A = spc.gather(plan, spc.ROWS, Asrc, 0, K, dt)
        B = spc.gather(plan, spc.COLS, Bsrc, 0, K, dt)
        out, Y = spc.sddmm_spmm(plan, vals, A, B, K)
        out_s = spc.sddmm(plan, vals, A, B, K)
        torch.cuda.synchronize()
        got = _np(out)[sample]
        caller = perm_np[sample]
        refs = [("fp32_inputs", p.A_src, p.B_src)]
        if name == "bf16":
            refs.append(("bf16_rounded_inputs", Ar, Br))
        for tag, Aref, Bref in refs:
            o, mo = oracle.sddmm(p.rows[caller], p.cols[caller], 0, 0, p.vals[caller], Aref, Bref,
                                 0, K)
            rel = 1e-5 if (name == "f32" or tag != "fp32_inputs") else E2E
            assert_within_mag(got, o, mo, rel, f"{name} sddmm vs {tag}")
            assert_within_mag(_np(out_s)[sample], o, mo, rel, f"{name} sddmm(sep) vs {tag}")
            report[f"{name}_sddmm_vs_{tag}"] = error_report(got, o, mo)
            pick, y, my = _sample_rows_oracle(p, np.random.default_rng(11), 2000, Bref, 0, K, 0)
            if tag == "fp32_inputs" and name == "f32":
                _say(f"  sampled rows include rows of up to "
                     f"{int(np.bincount(np.searchsorted(pick, p.rows[np.isin(p.rows, pick)])).max())}"
                     f" entries")
            loc = _np(m["lmap_r"])[pick - p.row_range[0]]
            gy = _np(Y[torch.from_numpy(loc).long().to(DEV)])
            assert_within_mag(gy, y, my, rel, f"{name} spmm vs {tag}")
            report[f"{name}_spmm_vs_{tag}"] = error_report(gy, y, my)
        # timing of the same calls (inputs resident, 5 back-to-back calls each)
        R, C, nnz, nb = plan.R, plan.C, p.nnz, (4 if name == "f32" else 2)
        alg = {"sddmm": 4 * (R + 1) + 12 * nnz + K * nb * (R + C),
               "spmm": 4 * (R + 1) + 8 * nnz + K * nb * C + 4 * K * R,
               "sddmm_spmm": 4 * (R + 1) + 12 * nnz + K * nb * (R + C) + 4 * K * R}
        calls = {"sddmm": lambda: spc.sddmm(plan, vals, A, B, K, out=out_s),
                 "spmm": lambda: spc.spmm(plan, vals, B, 0, K, out=Y),
                 "sddmm_spmm": lambda: spc.sddmm_spmm(plan, vals, A, B, K, out=out, Y=Y)}
        for op, fn in calls.items():
            ms = _time_ms(fn)
            report[f"{name}_{op}_time"] = {"ms": round(ms, 4), "GB_s": round(alg[op] / ms / 1e6, 1),
                                           "GFLOP_s": round((2 if op != "sddmm_spmm" else 4)
                                                            * K * nnz / ms / 1e6, 1)}
        del A, B, out, Y, out_s
        torch.cuda.empty_cache()
    print("PRECISION_REPORT " + json.dumps(report), flush=True)


def _time_ms(fn, reps=5):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps
