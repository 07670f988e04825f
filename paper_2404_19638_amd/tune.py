"""Exhaustive autotuner over the SDDMM / SpMM kernel variants.

A variant is (log2 lanes per nonzero, log2 of work-item slots / 64, wide SpMM batches).  The
autotuner times every valid variant of an operation on a plan with HIP events
on the current stream and returns the timings; it is the fallback of the
learned selector and the judge of its regret.
"""
from __future__ import annotations

import torch

from . import spc3d as spc

LG_LANES = (1, 2, 3, 4, 5, 6)
LG_ITEMS = (0, 1, 2, 3, 4)
ALL_VARIANTS = [spc.variant(a, b, w) for w in (0, 1) for a in LG_LANES for b in LG_ITEMS]
OPS = ("sddmm", "spmm", "sddmm_spmm")


def time_call(fn, reps: int = 20, warmup: int = 3) -> float:
    """Median milliseconds of fn() over reps, measured with events on the current stream."""
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return t[len(t) // 2]


def op_call(op: str, plan, vals, A, B, kz, variant, out, Y, buf):
    if op == "sddmm":
        return lambda: spc.sddmm(plan, vals, A, B, kz, out=out, variant=variant)
    if op == "spmm":
        return lambda: spc.spmm(plan, vals, B, 0, kz, out=Y, variant=variant, buf=buf)
    if op == "sddmm_spmm":
        return lambda: spc.sddmm_spmm(plan, vals, A, B, kz, out=out, Y=Y, variant=variant, buf=buf)
    raise ValueError(op)


def autotune(plan, op: str, vals, A, B, kz: int, variants=None, reps: int = 20) -> dict:
    """Time every valid variant of op; returns {variant: median ms} (invalid ones omitted)."""
    variants = ALL_VARIANTS if variants is None else variants
    dev = A.device
    out = torch.empty(plan.nnz, device=dev)
    Y = torch.empty((plan.R, kz), device=dev)
    buf = None
    res = {}
    for v in variants:
        try:
            if op != "sddmm":
                need = spc.spmm_buffer_size(plan, 0, kz, v)
                if buf is None or buf.numel() < need:
                    buf = torch.empty(need, dtype=torch.uint8, device=dev)
            fn = op_call(op, plan, vals, A, B, kz, v, out, Y, buf)
            fn()
        except spc.Spc3dError as e:
            if e.status in (spc.ERR_UNSUPPORTED, spc.ERR_INVALID_ARG):
                continue
            raise
        res[v] = time_call(fn, reps=reps)
    return res
