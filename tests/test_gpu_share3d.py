"""Parity on the benchmark workload at full size: one processor's 3D share of
an R-MAT graph (2^24 vertices, average degree 16, block (5,2) of the 8x8
grid, K-slice z = 1 of 4), the same block shape with uniform positions, and
a banded diagonal block of the same grid, run exactly as bench.py's step runs
it (gather A, gather B, fused SDDMM+SpMM, scatter-reduce; the library's
default shape and the variants the selector picks), against the FP64 oracle
on every output.

Integer and data-movement results are bit-exact; FP32 results lie within
1e-5 of the oracle's magnitude sum M elementwise.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth
from helpers import assert_within_mag

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # pragma: no cover - collected on CPU hosts too
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=["rmat", "uniform", "banded"])
def share(request):
    """The benchmark block (R-MAT), its uniform-position counterpart, and a
    banded diagonal block of the same grid."""
    p = {"rmat": synth.share3d, "uniform": synth.share3d_uniform,
         "banded": synth.share3d_banded}[request.param]()
    ref = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range)
    return p, ref


def test_share3d_step_full_size(share):
    from paper_2404_19638_amd import spc3d as spc
    p, ref = share
    _say(f"share3d nnz={p.nnz} R={ref['R']} C={ref['C']}")
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range)
    m = plan.maps()
    for k in ("gmap_r", "gmap_c", "lmap_r", "lmap_c", "rowptr", "colidx", "perm"):
        np.testing.assert_array_equal(_np(m[k]), ref[k], err_msg=k)
    k0, kz = p.k0, p.kz
    A_src = torch.from_numpy(p.A_src).to(DEV)
    B_src = torch.from_numpy(p.B_src).to(DEV)
    A = spc.gather(plan, spc.ROWS, A_src, k0, kz)
    B = spc.gather(plan, spc.COLS, B_src, k0, kz)
    np.testing.assert_array_equal(_np(A), oracle.gather_f32(ref["gmap_r"], p.row_range[0],
                                                            p.A_src, k0, kz))
    np.testing.assert_array_equal(_np(B), oracle.gather_f32(ref["gmap_c"], p.col_range[0],
                                                            p.B_src, k0, kz))
    vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, torch.from_numpy(p.vals).to(DEV))
    o_sd, m_sd = oracle.sddmm(p.rows, p.cols, p.row_range[0], p.col_range[0], p.vals, p.A_src,
                              p.B_src, k0, kz)
    o_sd, m_sd = o_sd[ref["perm"]], m_sd[ref["perm"]]
    o_sp, m_sp = oracle.spmm(p.rows, p.cols, p.row_range[0], p.col_range[0], ref["lmap_r"],
                             ref["R"], p.vals, p.B_src, k0, kz)
    # the default shape, the FP32 selector pick, and a windowed variant
    for v in (-1, spc.variant(3, 2), spc.variant(3, 0, 0, 1)):
        _say(f"share3d fused variant={v}")
        out, Y = spc.sddmm_spmm(plan, vals, A, B, kz, variant=v)
        assert_within_mag(_np(out), o_sd, m_sd, what=f"fused sddmm v={v}")
        assert_within_mag(_np(Y), o_sp, m_sp, what=f"fused spmm v={v}")
    _say("share3d unfused")
    assert_within_mag(_np(spc.sddmm(plan, vals, A, B, kz)), o_sd, m_sd, what="sddmm")
    Y = spc.spmm(plan, vals, B, 0, kz)
    assert_within_mag(_np(Y), o_sp, m_sp, what="spmm")
    # PostComm: the device's own Y rows added into the owner's slab, bit-exact
    dst = torch.from_numpy(p.A_src).to(DEV)
    want = p.A_src.copy()
    oracle.scatter_add_f32(ref["gmap_r"], p.row_range[0], _np(Y), want, k0)
    spc.scatter_reduce(plan, spc.ROWS, Y, dst, k0)
    np.testing.assert_array_equal(_np(dst).view(np.uint32), want.view(np.uint32))
    # the same PostComm folded into the fused pass (the step bench.py times):
    # the slab ends bit for bit as the oracle's FP32 addition of the fused
    # pass's own rows, and the SDDMM values are the fused pass's
    _say("share3d fused pass with the scatter-reduce folded in")
    out_f, Y_f = spc.sddmm_spmm(plan, vals, A, B, kz)
    want = p.A_src.copy()
    oracle.scatter_add_f32(ref["gmap_r"], p.row_range[0], _np(Y_f), want, k0)
    dst = torch.from_numpy(p.A_src).to(DEV)
    out_s = spc.sddmm_spmm_scatter(plan, vals, A, B, dst, k0, kz)
    np.testing.assert_array_equal(_np(dst).view(np.uint32), want.view(np.uint32))
    assert torch.equal(out_s.view(torch.int32), out_f.view(torch.int32))


def test_share3d_identities_full_size(share):
    """Properties that hold at any size, on the full benchmark block:
    sum_p SDDMM(S, A, B)_p = sum_{l,k} A_loc[l,k] * SpMM(S, B)[l,k] (both sides
    reduced in FP64 on the GPU, bar 1e-5 of the sum of |terms|), and the
    transpose symmetry SDDMM(S^T, B, A) = SDDMM(S, A, B) entry by entry,
    bit-exact (each dot product's reduction order depends on k only)."""
    from paper_2404_19638_amd import spc3d as spc
    p, ref = share
    dev_rows, dev_cols = torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV)
    plan = spc.plan_create_coo(dev_rows, dev_cols, p.row_range, p.col_range)
    k0, kz = p.k0, p.kz
    A = spc.gather(plan, spc.ROWS, torch.from_numpy(p.A_src).to(DEV), k0, kz)
    B = spc.gather(plan, spc.COLS, torch.from_numpy(p.B_src).to(DEV), k0, kz)
    vc = torch.from_numpy(p.vals).to(DEV)
    vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, vc)
    out, Y = spc.sddmm_spmm(plan, vals, A, B, kz)
    lhs = out.double().sum()
    rhs = (A.double() * Y.double()).sum()
    m = plan.maps()
    lr = torch.repeat_interleave(torch.arange(plan.R, device=DEV),
                                 (m["rowptr"][1:] - m["rowptr"][:-1]).long())
    mag = (vals.double().abs()[:, None] * A.double().abs()[lr]
           * B.double().abs()[m["colidx"].long()]).sum()
    _say(f"sum identity: {float(lhs):.6e} vs {float(rhs):.6e} (|terms| {float(mag):.3e})")
    assert abs(float(lhs - rhs)) <= 1e-5 * float(mag)
    # transpose symmetry, in caller order
    planT = spc.plan_create_coo(dev_cols, dev_rows, p.col_range, p.row_range)
    valsT = spc.permute_values(planT, spc.CALLER_TO_SLOT, vc)
    outT = spc.sddmm(planT, valsT, B, A, kz)
    a = spc.permute_values(plan, spc.SLOT_TO_CALLER, spc.sddmm(plan, vals, A, B, kz))
    b = spc.permute_values(planT, spc.SLOT_TO_CALLER, outT)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("kz,k0", [(16, 16), (128, 0)])
def test_share3d_other_kslices(share, kz, k0):
    """The step at the K-slice widths `bench.py --kz` times (Z = 8 and Z = 1 of
    the same grid), on the full blocks: packed rows and the scatter-reduce
    bit-exact, the fused pass's SDDMM and SpMM within 1e-5 of the oracle's
    magnitude sum on every output."""
    from paper_2404_19638_amd import spc3d as spc
    p, ref = share
    _say(f"share3d kz={kz} nnz={p.nnz}")
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range)
    A = spc.gather(plan, spc.ROWS, torch.from_numpy(p.A_src).to(DEV), k0, kz)
    B = spc.gather(plan, spc.COLS, torch.from_numpy(p.B_src).to(DEV), k0, kz)
    np.testing.assert_array_equal(_np(A), oracle.gather_f32(ref["gmap_r"], p.row_range[0],
                                                            p.A_src, k0, kz))
    np.testing.assert_array_equal(_np(B), oracle.gather_f32(ref["gmap_c"], p.col_range[0],
                                                            p.B_src, k0, kz))
    vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, torch.from_numpy(p.vals).to(DEV))
    out, Y = spc.sddmm_spmm(plan, vals, A, B, kz)
    o_sd, m_sd = oracle.sddmm(p.rows, p.cols, p.row_range[0], p.col_range[0], p.vals, p.A_src,
                              p.B_src, k0, kz)
    assert_within_mag(_np(out), o_sd[ref["perm"]], m_sd[ref["perm"]], what=f"sddmm kz={kz}")
    del o_sd, m_sd
    o_sp, m_sp = oracle.spmm(p.rows, p.cols, p.row_range[0], p.col_range[0], ref["lmap_r"],
                             ref["R"], p.vals, p.B_src, k0, kz)
    assert_within_mag(_np(Y), o_sp, m_sp, what=f"spmm kz={kz}")
    dst = torch.from_numpy(p.A_src).to(DEV)
    want = p.A_src.copy()
    oracle.scatter_add_f32(ref["gmap_r"], p.row_range[0], _np(Y), want, k0)
    spc.scatter_reduce(plan, spc.ROWS, Y, dst, k0)
    np.testing.assert_array_equal(_np(dst).view(np.uint32), want.view(np.uint32))
