"""Calls on several HIP streams at once (default stream priority throughout).

The library keeps no per-call state of its own besides the arguments (the
static scratch of spc3d_sddmm_spmm_static and the plan checker's word aside,
documented as shared per GPU), so two plans driven from two streams
concurrently, and one plan driven from two streams with a buffer and outputs
per stream, must give, bit for bit, what the same calls give one after
another."""
import sys

import pytest

from paper_2404_19638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _case(spc, seed, kind):
    if kind == "rmat":
        p = synth.small_rmat(14, 8, 32, seed, row_range=(1 << 13, 1 << 14), col_range=(0, 1 << 13))
        rows, cols, rr, cr = p.rows, p.cols, p.row_range, p.col_range
    else:
        rows, cols = synth.uniform_block(20000, 30000, 300_000, seed)
        rr, cr = (0, 20000), (0, 30000)
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               rr, cr)
    kz = 32
    A = torch.from_numpy(synth.dense_f32(seed + 1, 0, plan.R, kz)).to(DEV)
    B = torch.from_numpy(synth.dense_f32(seed + 2, 0, plan.C, kz)).to(DEV)
    v = torch.from_numpy(synth.uniform_f32(seed + 3, plan.nnz)).to(DEV)
    return plan, A, B, v, kz


def _outs(spc, plan, kz):
    return (torch.empty(plan.nnz, device=DEV), torch.empty((plan.R, kz), device=DEV),
            torch.empty(spc.spmm_buffer_size(plan, 0, kz), dtype=torch.uint8, device=DEV))


def _bits(t):
    return t.view(torch.int32)


def test_two_plans_on_two_streams():
    spc = _spc()
    cases = [_case(spc, 11, "rmat"), _case(spc, 12, "uniform")]
    want = []
    for plan, A, B, v, kz in cases:
        o, Y = spc.sddmm_spmm(plan, v, A, B, kz)
        want.append((o.clone(), Y.clone()))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [_outs(spc, c[0], c[4]) for c in cases]
    torch.cuda.synchronize()
    _say("streams: two plans, two streams, 8 rounds")
    for _ in range(8):
        for (plan, A, B, v, kz), s, (o, Y, buf) in zip(cases, streams, outs):
            with torch.cuda.stream(s):
                spc.sddmm_spmm(plan, v, A, B, kz, out=o, Y=Y, buf=buf)
    torch.cuda.synchronize()
    for (o, Y, _), (wo, wY) in zip(outs, want):
        assert torch.equal(_bits(o), _bits(wo)) and torch.equal(_bits(Y), _bits(wY))


def test_one_plan_on_two_streams_with_a_buffer_each():
    spc = _spc()
    plan, A, B, v, kz = _case(spc, 21, "rmat")
    wo, wY = spc.sddmm_spmm(plan, v, A, B, kz)
    wo, wY = wo.clone(), wY.clone()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [_outs(spc, plan, kz) for _ in streams]
    torch.cuda.synchronize()
    _say("streams: one plan, two streams, 8 rounds")
    for _ in range(8):
        for s, (o, Y, buf) in zip(streams, outs):
            with torch.cuda.stream(s):
                spc.sddmm_spmm(plan, v, A, B, kz, out=o, Y=Y, buf=buf)
    torch.cuda.synchronize()
    for o, Y, _ in outs:
        assert torch.equal(_bits(o), _bits(wo)) and torch.equal(_bits(Y), _bits(wY))
