"""Exhaustive autotuner over the SDDMM / SpMM kernel variants.

A variant is (log2 lanes per nonzero, log2 of work-item slots / 64, wide SpMM
batches), encoded by ``spc3d.variant``.  The autotuner times every valid
variant of an operation on a plan with HIP events on the current stream and
returns the timings; it is the fallback of the learned selector and the judge
of its regret.
"""
from __future__ import annotations

import torch

from . import spc3d as spc

LG_LANES = (1, 2, 3, 4, 5, 6)
LG_ITEMS = (0, 1, 2, 3, 4)
# group-run SpMM family (8- or 16-row batches), then the windowed family
GROUP_VARIANTS = [spc.variant(a, b, w) for w in (0, 1) for a in LG_LANES for b in LG_ITEMS]
WINDOW_VARIANTS = [spc.variant(a, b, 0, 1) for a in (1, 2, 3) for b in LG_ITEMS]
ALL_VARIANTS = GROUP_VARIANTS + WINDOW_VARIANTS
OPS = ("sddmm", "spmm", "sddmm_spmm")
OPCODE = {"sddmm": spc.OP_SDDMM, "spmm": spc.OP_SPMM, "sddmm_spmm": spc.OP_SDDMM_SPMM}


def candidates(op: str) -> list:
    """Variants that differ for op: the SDDMM kernel ignores the SpMM bits."""
    if op == "sddmm":
        return [v for v in ALL_VARIANTS if not (v >> 8) & 3]
    return list(ALL_VARIANTS)


def valid(op: str, kz: int, dtype: int, variant: int) -> bool:
    return spc.variant_check(OPCODE[op], kz, dtype, variant) == spc.OK


_sleep_cycles_per_ms = None


def _spacer(ms: float):
    """Queue a spin kernel of about ms milliseconds, so that the calls queued
    after it run back to back instead of waiting for the host."""
    global _sleep_cycles_per_ms
    if _sleep_cycles_per_ms is None:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(1000)
        a.record()
        torch.cuda._sleep(1_000_000)
        b.record()
        torch.cuda.synchronize()
        _sleep_cycles_per_ms = 1_000_000 / max(a.elapsed_time(b), 1e-3)
    torch.cuda._sleep(max(1000, int(ms * _sleep_cycles_per_ms)))


def time_call(fn, reps: int = 5, warmup: int = 1, batches: int = 1) -> float:
    """Milliseconds per call of fn(): the least, over batches, of the mean of
    reps back-to-back calls timed with events on the current stream."""
    for _ in range(warmup):
        fn()
    best = None
    for _ in range(batches):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        _spacer(0.05 * reps + 0.1)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) / reps
        best = t if best is None else min(best, t)
    return best


def op_call(op: str, plan, vals, A, B, kz, variant, out, Y, buf):
    if op == "sddmm":
        return lambda: spc.sddmm(plan, vals, A, B, kz, out=out, variant=variant)
    if op == "spmm":
        return lambda: spc.spmm(plan, vals, B, 0, kz, out=Y, variant=variant, buf=buf)
    if op == "sddmm_spmm":
        return lambda: spc.sddmm_spmm(plan, vals, A, B, kz, out=out, Y=Y, variant=variant, buf=buf)
    raise ValueError(op)


def autotune(plan, op: str, vals, A, B, kz: int, variants=None, reps: int = 5,
             batches: int = 1) -> dict:
    """Time every valid variant of op (and -1, the default shape); returns
    {variant: ms per call}, invalid variants omitted."""
    variants = [-1] + candidates(op) if variants is None else variants
    dev = A.device
    out = torch.empty(plan.nnz, device=dev)
    Y = torch.empty((plan.R, kz), device=dev)
    buf = None
    res = {}
    warm = True
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
        if warm:
            # one untimed round of the first runnable variant, as it will be
            # timed: otherwise the first variant of each instance is timed
            # slower than the same shape timed later (by up to 4% on MI355X)
            time_call(fn, reps=reps, warmup=0, batches=1)
            warm = False
        res[v] = time_call(fn, reps=reps, warmup=0, batches=batches)
    return res


def best_variant(timings: dict) -> int:
    """The fastest variant of an autotune result (the default on an empty one)."""
    return min(timings, key=lambda v: (timings[v], v)) if timings else -1
