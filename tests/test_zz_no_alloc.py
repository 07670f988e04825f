"""spc3d_sddmm_spmm_static, the fused pass for callers that cannot allocate:
its outputs against spc3d_sddmm_spmm's (the same kernels with a caller
buffer) bit for bit, and against the FP64 oracle at 1e-5 M, on two calls in
a row, the second on a smaller block; a call whose carries exceed the static
scratch is refused before any launch."""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth
from helpers import assert_within_mag

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _case(spc, scale, seed, kz, dtype):
    p = synth.small_rmat(scale, 8, 64, seed, row_range=(1 << (scale - 1), 1 << scale),
                         col_range=(0, 1 << (scale - 1)))
    ref = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range)
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range)
    k0 = 64 - kz
    A = spc.gather(plan, spc.ROWS, torch.from_numpy(p.A_src).to(DEV), k0, kz, dtype)
    B = spc.gather(plan, spc.COLS, torch.from_numpy(p.B_src).to(DEV), k0, kz, dtype)
    v = torch.from_numpy(p.vals[ref["perm"]]).to(DEV)
    return p, ref, plan, A, B, v, k0


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_static_scratch_matches_buffered_entry_point(dtype):
    spc = __import__("paper_2404_19638_amd.spc3d", fromlist=["spc3d"])
    kz = 32
    for step, scale in enumerate((16, 11)):   # the second call on a smaller block
        p, ref, plan, A, B, v, k0 = _case(spc, scale, 60 + scale, kz, dtype)
        _say(f"static scratch call {step}: {dtype} nnz={plan.nnz} kz={kz}")
        out = torch.empty(plan.nnz, device=DEV)
        Y = torch.empty((plan.R, kz), device=DEV)
        spc.sddmm_spmm_static(plan, v, A, B, kz, out=out, Y=Y)
        want_out, want_Y = spc.sddmm_spmm(plan, v, A, B, kz)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical bits
        assert torch.equal(out, want_out) and torch.equal(Y, want_Y)
        if dtype == torch.float32:
            Asrc, Bsrc = p.A_src, p.B_src
        else:
            Asrc = oracle.bf16_to_f32(oracle.bf16_rne(p.A_src))
            Bsrc = oracle.bf16_to_f32(oracle.bf16_rne(p.B_src))
        o, mo = oracle.sddmm(p.rows, p.cols, p.row_range[0], p.col_range[0], p.vals, Asrc, Bsrc,
                             k0, kz)
        assert_within_mag(_np(out), o[ref["perm"]], mo[ref["perm"]], what="static sddmm")
        y, my = oracle.spmm(p.rows, p.cols, p.row_range[0], p.col_range[0], ref["lmap_r"],
                            ref["R"], p.vals, Bsrc, k0, kz)
        assert_within_mag(_np(Y), y, my, what="static spmm")
        # ACCUMULATE adds this call's result to what the outputs hold
        spc.sddmm_spmm_static(plan, v, A, B, kz, out=out, Y=Y, mode=spc.ACCUMULATE)
        spc.sddmm_spmm(plan, v, A, B, kz, out=want_out, Y=want_Y, mode=spc.ACCUMULATE)
        torch.cuda.synchronize()
        assert torch.equal(out, want_out) and torch.equal(Y, want_Y)


def test_static_scratch_refuses_oversize_calls():
    spc = __import__("paper_2404_19638_amd.spc3d", fromlist=["spc3d"])
    kz = 1024
    p = synth.small_rmat(15, 8, 64, 75, row_range=(0, 1 << 15), col_range=(0, 1 << 15))
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range)
    _say(f"static scratch oversize: nnz={plan.nnz} kz={kz}")
    assert spc.spmm_buffer_size(plan, 0, kz) > spc.STATIC_SCRATCH_BYTES
    A = torch.zeros((plan.R, kz), device=DEV)
    B = torch.zeros((plan.C, kz), device=DEV)
    out = torch.full((plan.nnz,), 7.0, device=DEV)
    Y = torch.full((plan.R, kz), 7.0, device=DEV)
    with pytest.raises(spc.Spc3dError) as e:
        spc.sddmm_spmm_static(plan, None, A, B, kz, out=out, Y=Y)
    assert e.value.status == spc.ERR_WORKSPACE
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    # nothing was launched: the outputs are untouched
    assert bool((out == 7.0).all()) and bool((Y == 7.0).all())
