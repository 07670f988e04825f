"""Benchmark of the local SDDMM + SpMM hot path on one MI355X.

One step = one iteration of the paper's per-iteration loop on one processor's
share (PreComm local side, Compute, PostComm local side):
    gather A rows -> gather B rows -> SDDMM -> SpMM -> scatter-reduce
over a localized block built once beforehand (the setup phase, timed and
reported separately).  By default SDDMM and SpMM run as one pass followed by
the scatter-reduce; --fused 2 folds the scatter-reduce into the pass (each
SpMM row added into the owner's slab as it completes, bit-identical) and
--fused 0 runs every step separately.  All three forms are timed and
reported under step_forms.  Default workload: one processor's 3D share of an R-MAT
graph (2^24 vertices, average degree 16) on an 8x8x4 grid, i.e. a 2^21 x 2^21
block with ~4M entries, K = 128 and the local K-slice kz = 32, FP32.

Prints one JSON line.  ``value`` is SDDMM + SpMM GFLOP/s (2*kz*nnz flops each)
over the whole step time with inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources of the step's kernels and of the slot structure they read (the
# setup): the recorded traffic of a kernel is valid while these are unchanged.
STEP_SOURCES = ("internal.h", "vec.h", "kernels.h", "compute.hip", "pack.hip", "plan.hip",
                "inst_fused_f32.hip", "inst_fused_bf16.hip", "inst_sddmm_f32.hip",
                "inst_sddmm_bf16.hip", "inst_spmm_f32.hip", "inst_spmm_bf16.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2404_19638_amd", "csrc")
    for f in STEP_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(R, C, nnz, kz, b):
    """Compulsory HBM bytes per launch: each input read once, each output written once."""
    return {
        "gather_A": 8 * R + (4 + b) * kz * R,
        "gather_B": 8 * C + (4 + b) * kz * C,
        "sddmm": 4 * (R + 1) + 12 * nnz + kz * b * (R + C),
        "spmm": 4 * (R + 1) + 8 * nnz + kz * b * C + 4 * kz * R,
        "scatter": 8 * R + 12 * kz * R,
        # one pass: S structure, values and B rows read once for both products
        "sddmm_spmm": 4 * (R + 1) + 12 * nnz + kz * b * (R + C) + 4 * kz * R,
        # the same pass adding each row into the owner's slab: the slab rows
        # read and written, and the row map, in place of the packed Y
        "sddmm_spmm_scatter": 4 * (R + 1) + 12 * nnz + kz * b * (R + C) + 8 * R + 8 * kz * R,
    }


def load_traffic(kernel: str, workload: str, src_hash: str):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        e = t.get(f"{workload}:{kernel}")
        if e and e.get("source_hash") == src_hash:
            return e.get("bytes_per_launch")
    except (OSError, ValueError):
        pass
    return None


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or 'unknown'."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, budget_s=12.0):
    """The FP64 oracle (as it stands, single-threaded) on the same workload."""
    import numpy as np
    import oracle

    t0 = time.perf_counter()
    ref = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range)
    t_setup = time.perf_counter() - t0
    k0, kz = p.k0, p.kz
    dst = np.zeros((p.row_range[1] - p.row_range[0], p.K), np.float32)
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 50:
        t0 = time.perf_counter()
        oracle.gather_f32(ref["gmap_r"], p.row_range[0], p.A_src, k0, kz)
        oracle.gather_f32(ref["gmap_c"], p.col_range[0], p.B_src, k0, kz)
        oracle.sddmm(p.rows, p.cols, p.row_range[0], p.col_range[0], p.vals, p.A_src, p.B_src,
                     k0, kz)
        y, _ = oracle.spmm(p.rows, p.cols, p.row_range[0], p.col_range[0], ref["lmap_r"],
                           ref["R"], p.vals, p.B_src, k0, kz)
        oracle.scatter_add_f32(ref["gmap_r"], p.row_range[0], y.astype(np.float32), dst, k0)
        t_total += time.perf_counter() - t0
        reps += 1
    t_step = t_total / reps
    flops = 4.0 * kz * p.nnz
    return {"value": round(flops / t_step / 1e9, 4), "unit": "GFLOP/s", "cores": 1,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": (f"the full workload: {reps} oracle steps (gather A, gather B, SDDMM, SpMM, "
                       f"scatter-reduce in FP64, one thread) on the same block, "
                       f"{t_step * 1e3:.1f} ms per step; oracle localization {t_setup:.2f} s")}


ERROR_BARS = {
    "f32": "|x - x*| <= 1e-5 M elementwise vs the FP64 oracle (M = sum of |terms|)",
    "bf16": "|x - x*| <= (2^-7 + 2^-16 + 1e-5) M vs the FP64 oracle on the FP32 inputs; "
            "<= 1e-5 M vs the oracle on the BF16-rounded inputs",
}
SELECTOR_WEIGHTS = os.path.join(ROOT, "paper_2404_19638_amd", "selector_weights.json")


def copy_bandwidth(dev, mib=1024, reps=10):
    """GB/s of a plain device-to-device copy of `mib` MiB (read + write bytes)."""
    import torch
    n = mib << 18
    a = torch.ones(n, device=dev)
    c = torch.empty_like(a)
    for _ in range(2):
        c.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        c.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, c
    torch.cuda.empty_cache()
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def cold_steps(step, names, spans, nev, alg, steps, dev, flops, dirty=False):
    """The step and each kernel with L2 and the Infinity Cache flushed before
    every step (the flush is outside the events, which bracket the step from
    its first kernel to its last).  The flush writes 1 GiB, which evicts the
    step's lines, then reads it back, so that the cache holds clean lines
    and the step does not also pay for writing the flush's dirty lines back
    to HBM.  dirty=True leaves out the read: the step then runs against a
    cache full of dirty lines."""
    import numpy as np
    import torch

    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    sink = torch.empty(1, dtype=torch.float32, device=dev)
    evs = []
    for i in range(steps):
        flush.fill_(float(i))
        if not dirty:
            torch.sum(flush, 0, keepdim=True, out=sink)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(nev)]
        step(ev)
        evs.append(ev)
    torch.cuda.synchronize()
    kernels = {}
    for n in names:
        a, b = spans[n]
        ms = float(np.mean([e[a].elapsed_time(e[b]) for e in evs]))
        kernels[n] = {"ms": round(ms, 5), "GB_s": round(alg[n] / (ms * 1e-3) / 1e9, 1),
                      "frac_hbm": round(alg[n] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    step_ms = float(np.mean([e[0].elapsed_time(e[nev - 1]) for e in evs]))
    total = sum(alg[n] for n in names)
    dom = max(names, key=lambda n: kernels[n]["ms"])
    del flush
    return {"steps": steps, "flush": "1 GiB write" if dirty else "1 GiB write, then read",
            "step_ms": round(step_ms, 5),
            "value": round(flops / (step_ms * 1e-3) / 1e9, 2),
            "step_frac_hbm": round(total / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": kernels[dom]["GB_s"],
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kernels[dom]["frac_hbm"]},
            "kernels": kernels}


def forms(args, spc, plan, kz, nnz, make_step, timed, names, ms_main, per_main, flops):
    """The plain FP32 form against BF16 operands and the learned selector's
    variants, each timed like the main loop on the same block."""
    import torch

    sel = None
    if os.path.exists(SELECTOR_WEIGHTS):
        from paper_2404_19638_amd.selector import Selector, load_weights
        sel = Selector.from_state(load_weights(SELECTOR_WEIGHTS), plan.ws.device)
    out = {}
    for dt in ("f32", "bf16"):
        code = spc.F32 if dt == "f32" else spc.BF16
        entries = [("default", -1, "library default shape")]
        if sel is not None:
            tdt = torch.float32 if dt == "f32" else torch.bfloat16
            A = torch.rand((plan.R, kz), device=plan.ws.device).to(tdt)
            B = torch.rand((plan.C, kz), device=plan.ws.device).to(tdt)
            if args.fused:
                v, src = sel.choose(plan, "sddmm_spmm", kz, code, A=A, B=B)
            else:
                v1, s1 = sel.choose(plan, "sddmm", kz, code, A=A, B=B)
                v2, s2 = sel.choose(plan, "spmm", kz, code, A=A, B=B)
                v, src = (v1, v2), f"{s1}/{s2}"
            entries.append(("learned", v, f"selector ({src})"))
        measured = {}
        for tag, v, how in entries:
            key = v if isinstance(v, int) else tuple(v)
            if dt == args.dtype and v == args.variant:
                ms, per = ms_main, per_main
            elif key in measured:   # the selector kept the default: the same step, timed once
                ms, per = measured[key]
            else:
                ms, per = timed(make_step(dt, v), args.steps, args.warmup)
            measured[key] = (ms, per)
            dom = max(names, key=lambda n: per[n])
            out[f"{dt}_{tag}"] = {"variant": list(v) if isinstance(v, tuple) else v,
                                  "chosen_by": how, "ms_per_step": round(ms, 5),
                                  "value": round(flops / (ms * 1e-3) / 1e9, 2),
                                  "compute_kernel_ms": round(sum(per[n] for n in names
                                                                 if not n.startswith("gather")
                                                                 and n != "scatter"), 5),
                                  "dominant": dom, "error_bar": ERROR_BARS[dt]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cold-steps", type=int, default=10,
                    help="extra steps, each after a 1 GiB flush, for cold-cache step and kernel times")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the BF16 and learned-selector forms")
    ap.add_argument("--seed", type=int, default=2405)
    ap.add_argument("--kz", type=int, default=0,
                    help="K-slice width of the 3D-share blocks (K = 128; Z = K / kz processors "
                         "along the third grid axis); default 32, i.e. Z = 4")
    ap.add_argument("--graph", action="store_true",
                    help="time the K steps as replays of one step captured in a HIP graph "
                         "(both are always measured and reported under 'launch')")
    ap.add_argument("--fused", type=int, default=1, choices=[0, 1, 2],
                    help="2: one pass for SDDMM, SpMM and the scatter-reduce; 1: a fused "
                         "SDDMM+SpMM pass and the scatter-reduce; 0: separate kernels")
    ap.add_argument("--workload", choices=["share3d", "uniform", "banded", "tiny", "precision"],
                    default="share3d",
                    help="share3d: one processor's block of R-MAT 2^24 (the benchmark); "
                         "uniform: the same block shape with uniform positions; "
                         "banded: a diagonal block of the same grid with a banded pattern; "
                         "tiny: 4096^2 with 40,000 uniform entries, K = 32 (latency-bound); "
                         "precision: R-MAT 2^22, degree 32, whole matrix, K = kz = 128")
    ap.add_argument("--row-groups", type=int, default=0, metavar="G",
                    help="owner-grouped local rows (SpC-RB order): seeded keys in [0, G)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: spc3d has no exchange "
                                   "between GPUs (the path would shard one block of the 3D "
                                   "grid per GPU)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2404_19638_amd import spc3d as spc
    from paper_2404_19638_amd import synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        n = args.calibrate_copy << 18
        a = torch.ones(n, device=dev)
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        del a, c
    t0 = time.perf_counter()
    p = {"share3d": lambda: synth.share3d(seed=args.seed), "tiny": synth.tiny,
         "uniform": synth.share3d_uniform, "banded": synth.share3d_banded,
         "precision": synth.precision}[args.workload]()
    log(f"bench: generated {args.workload} block nnz={p.nnz} in {time.perf_counter() - t0:.1f} s")
    if args.kz:
        if args.workload not in ("share3d", "uniform", "banded") or p.K % args.kz:
            raise SystemExit("--kz applies to the 3D-share blocks (K = 128) and must divide K")
        p.kz, p.k0 = args.kz, args.kz * (1 if args.kz < p.K else 0)   # the slice z = 1 (or 0)
    zdim = p.K // p.kz
    rows = torch.from_numpy(p.rows).to(dev)
    cols = torch.from_numpy(p.cols).to(dev)
    A_src = torch.from_numpy(p.A_src).to(dev)
    B_src = torch.from_numpy(p.B_src).to(dev)
    Y_dst = torch.zeros_like(A_src)
    vals_caller = torch.from_numpy(p.vals).to(dev)
    torch.cuda.synchronize()

    # setup phase (once per pattern), timed separately
    t0 = time.perf_counter()
    groups = {}
    if args.row_groups:
        rr = p.row_range[1] - p.row_range[0]
        keys = (synth.draws_u64(args.seed + 3, rr) % np.uint64(args.row_groups)).astype(np.int32)
        groups = dict(group_r=torch.from_numpy(keys).to(dev), ngroups_r=args.row_groups)
    plan = spc.plan_create_coo(rows, cols, p.row_range, p.col_range, **groups)
    vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, vals_caller)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    R, C, nnz, kz, k0 = plan.R, plan.C, plan.nnz, p.kz, p.k0
    # the same setup again in the workspace the first call allocated: the
    # first call also pays the allocation and the first launch of each kernel
    ws, warm = plan.ws, []
    for _ in range(5):
        del plan
        t0 = time.perf_counter()
        plan = spc.plan_create_coo(rows, cols, p.row_range, p.col_range, ws=ws, **groups)
        vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, vals_caller)
        torch.cuda.synchronize()
        warm.append((time.perf_counter() - t0) * 1e3)
    setup_warm_ms = float(np.median(warm))
    log(f"bench: plan R={R} C={C} nnz={nnz} setup {setup_ms:.1f} ms (first), "
        f"{setup_warm_ms:.2f} ms (again)")

    # Events: 0 start, 1 after gather A, 2 / 3 around gather B, 4 start of the
    # compute, then one after each remaining kernel.  (Running the two packs on
    # two streams was measured slower than one after the other: they contend
    # for the same HBM bandwidth.)
    def layout(kind):
        """Kernels of a step form, kernel -> (start event, end event), event count."""
        spans = {"gather_A": (0, 1), "gather_B": (2, 3)}
        if kind == 2:
            spans.update(sddmm_spmm_scatter=(4, 5))
        elif kind == 1:
            spans.update(sddmm_spmm=(4, 5), scatter=(5, 6))
        else:
            spans.update(sddmm=(4, 5), spmm=(5, 6), scatter=(6, 7))
        return list(spans), spans, len(spans) + 3

    names, spans, nev = layout(args.fused)

    def make_step(dtype, variant, kind=None):
        """One step in dtype; variant is an int, or (SDDMM, SpMM) variants when unfused;
        kind the step form (default --fused).  step(ev) records events ev[0..nev)."""
        kind = args.fused if kind is None else kind
        last = layout(kind)[2] - 1
        v_sd, v_sp = variant if isinstance(variant, tuple) else (variant, variant)
        pdt = torch.float32 if dtype == "f32" else torch.bfloat16
        A_loc = torch.empty((R, kz), dtype=pdt, device=dev)
        B_loc = torch.empty((C, kz), dtype=pdt, device=dev)
        out = torch.empty(nnz, device=dev)
        Y_loc = torch.empty((R, kz), device=dev)
        spbuf = torch.empty(spc.spmm_buffer_size(plan, 0, kz, v_sp), dtype=torch.uint8,
                            device=dev)

        def step(ev=None):
            def mark(i):
                if ev is not None:
                    ev[i].record()
            mark(0)
            spc.gather(plan, spc.ROWS, A_src, k0, kz, out=A_loc)
            mark(1)
            mark(2)
            spc.gather(plan, spc.COLS, B_src, k0, kz, out=B_loc)
            mark(3)
            mark(4)
            if kind == 2:
                spc.sddmm_spmm_scatter(plan, vals, A_loc, B_loc, Y_dst, k0, kz, out=out,
                                       variant=v_sp, buf=spbuf)
            elif kind == 1:
                spc.sddmm_spmm(plan, vals, A_loc, B_loc, kz, out=out, Y=Y_loc, variant=v_sp,
                               buf=spbuf)
                mark(5)
                spc.scatter_reduce(plan, spc.ROWS, Y_loc, Y_dst, k0)
            else:
                spc.sddmm(plan, vals, A_loc, B_loc, kz, out=out, variant=v_sd)
                mark(5)
                spc.spmm(plan, vals, B_loc, 0, kz, out=Y_loc, variant=v_sp, buf=spbuf)
                mark(6)
                spc.scatter_reduce(plan, spc.ROWS, Y_loc, Y_dst, k0)
            mark(last)
        return step

    spread = {}   # kernel -> (median, min) ms of the last timed() call

    def timed(step, steps, warmup, kind=None):
        """Step time from exactly `steps` steps with nothing recorded between them
        (the timing markers of the per-kernel pass add gaps between kernels), then
        per-kernel times from a second pass with events around every kernel
        (every event pair is on the stream the kernels run on)."""
        _, spans_k, nev_k = layout(args.fused if kind is None else kind)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        events = [[torch.cuda.Event(enable_timing=True) for _ in range(nev_k)]
                  for _ in range(steps)]
        for i in range(steps):
            step(events[i])
        torch.cuda.synchronize()
        samples = {n: [events[i][a].elapsed_time(events[i][b]) for i in range(steps)]
                   for n, (a, b) in spans_k.items()}
        per = {n: float(np.mean(v)) for n, v in samples.items()}
        spread.clear()
        spread.update({n: (float(np.median(v)), float(np.min(v))) for n, v in samples.items()})
        return ms, per

    def graph_timed(step, steps, warmup):
        """Step time from `steps` replays of one step captured in a HIP graph
        (the same kernels on the same buffers, without per-launch host work)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        del g
        return ms

    b = 4 if args.dtype == "f32" else 2
    main_step = make_step(args.dtype, args.variant)
    eager_ms, per_kernel_ms = timed(main_step, args.steps, args.warmup)
    per_kernel_spread = dict(spread)
    graph_ms = graph_timed(main_step, args.steps, args.warmup)
    ms_per_step = graph_ms if args.graph else eager_ms
    flops = 4.0 * kz * nnz
    value = flops / (ms_per_step * 1e-3) / 1e9
    alg = algorithmic_bytes(R, C, nnz, kz, b)
    dominant = max(names, key=lambda n: per_kernel_ms[n])
    achieved = alg[dominant] / (per_kernel_ms[dominant] * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    workload = {"share3d": f"rmat24-deg16-block(5,2)-8x8x{zdim}-kz{kz}",
                "uniform": f"uniform-block(5,2)-8x8x{zdim}-kz{kz}-4012517nnz",
                "banded": f"banded-hw16384-block(2,2)-8x8x{zdim}-kz{kz}",
                "tiny": "uniform-4096x4096-40000nnz-k32",
                "precision": "rmat22-deg32-whole-k128"}[args.workload]
    kernels = {n: {"ms": round(per_kernel_ms[n], 5),
                   "ms_median": round(per_kernel_spread[n][0], 5),
                   "ms_min": round(per_kernel_spread[n][1], 5), "alg_bytes": int(alg[n]),
                   "GB_s": round(alg[n] / (per_kernel_ms[n] * 1e-3) / 1e9, 1),
                   "frac_hbm": round(alg[n] / (per_kernel_ms[n] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
               for n in names}
    total_alg = sum(alg[n] for n in names)
    copy_gbs = copy_bandwidth(dev)
    for n in names:
        kernels[n]["frac_copy"] = round(kernels[n]["GB_s"] / copy_gbs, 4)
    res = {
        "metric": "SDDMM+SpMM GFLOP/s",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "f32" else "bf16-in/f32-acc",
        "data": "synthetic (seeded R-MAT stand-in for the paper's SuiteSparse graphs)",
        "config": {"workload": workload,
                   **({"rmat_scale": 24, "avg_degree": 16, "grid": f"8x8x{zdim}", "block": [5, 2]}
                      if args.workload == "share3d" else
                      {"grid": f"8x8x{zdim}", "block": [5, 2]} if args.workload == "uniform" else
                      {"grid": f"8x8x{zdim}", "block": [2, 2], "band_half_width": 16384,
                       "draws_per_row": 2} if args.workload == "banded" else
                      {"rmat_scale": 22, "avg_degree": 32, "grid": "1x1x1"}
                      if args.workload == "precision" else {"grid": "1x1x1"}),
                   "R": R, "C": C, "nnz": nnz, "K": p.K, "kz": kz, "k0": k0,
                   "step": {2: "gather A, gather B, one pass of SDDMM+SpMM with the "
                                "scatter-reduce folded in",
                            1: "gather A, gather B, fused SDDMM+SpMM, scatter-reduce",
                            0: "gather A, gather B, SDDMM, SpMM, scatter-reduce"}[args.fused],
                   "local_row_order": (f"owner-grouped, {args.row_groups} groups"
                                       if args.row_groups else "ascending global id")},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(dominant, workload, src_hash)},
        "step_frac_hbm": round(total_alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_GB_s": round(copy_gbs, 1),
        "step_frac_copy": round(total_alg / (ms_per_step * 1e-3) / 1e9 / copy_gbs, 4),
        "kernels": kernels,
        "launch": {"timed_steps": "hip graph replays" if args.graph else "eager launches",
                   "eager_ms_per_step": round(eager_ms, 5),
                   "graph_ms_per_step": round(graph_ms, 5)},
        "setup_ms": round(setup_ms, 2),
        "setup_warm_ms": round(setup_warm_ms, 3),
        "source_hash": src_hash,
    }
    # the other forms of the same step (the same results; the scatter-reduce
    # folded into the pass, or each kernel on its own)
    res["step_forms"] = {}
    for kind in (2, 1, 0):
        if kind == args.fused:
            ms_k = ms_per_step
        else:
            ms_k, _ = timed(make_step(args.dtype, args.variant, kind), args.steps, args.warmup,
                            kind)
        res["step_forms"][{2: "scatter_folded", 1: "fused_then_scatter", 0: "separate"}[kind]] = {
            "ms_per_step": round(ms_k, 5), "value": round(flops / (ms_k * 1e-3) / 1e9, 2)}
    if args.cold_steps:
        res["cold"] = cold_steps(make_step(args.dtype, args.variant), names, spans, nev, alg,
                                 args.cold_steps, dev, flops)
        d = cold_steps(make_step(args.dtype, args.variant), names, spans, nev, alg,
                       args.cold_steps, dev, flops, dirty=True)
        res["cold"]["dirty_flush"] = {"flush": d["flush"], "step_ms": d["step_ms"],
                                      "value": d["value"],
                                      "kernels_ms": {n: d["kernels"][n]["ms"] for n in names}}
    if not args.no_forms:
        res["forms"] = forms(args, spc, plan, kz, nnz, make_step, timed, names, eager_ms,
                             per_kernel_ms, flops)
    if not args.no_cpu:
        log("bench: timing the CPU oracle baseline")
        res["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
