"""The fused pass with the SpMM PostComm folded in (spc3d_sddmm_spmm_scatter):
each row sum is added into the owner's slab once, as it completes, so the
slab must end bit for bit as the FP64 oracle's FP32 addition of the rows the
plain fused pass produces (oracle_scatter_add_f32), and the SDDMM values must
equal the plain fused pass's.  Covered: the default shape and each SpMM
family, FP32 and bfloat16 operands, out in OVERWRITE and ACCUMULATE, rows cut
by work items (the carry fix-up), a column offset off 16-byte alignment (the
scalar shape), an owner-grouped local order, and the argument checks."""
import sys

import numpy as np
import pytest

import oracle
from paper_2404_19638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _np(t):
    return t.detach().cpu().numpy()


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint32)


def _check(spc, plan, gmap_r, row_lo, vals, A, B, dst_np, k0, kz, variant, out_mode, tag):
    """sddmm_spmm_scatter against sddmm_spmm + oracle scatter-add, bit for bit.
    The plain pass writes its rows with the same alignment as the slab's rows
    (k0 off a multiple of 4 takes the scalar shape in both), so both run the
    same kernel shape and sum every row in the same order."""
    if k0 % 4:
        ybuf = torch.empty(plan.R * kz + 4, device=DEV)
        Y_f = ybuf[k0 % 4:k0 % 4 + plan.R * kz].view(plan.R, kz)
    else:
        Y_f = None
    out_f, Y_f = spc.sddmm_spmm(plan, vals, A, B, kz, Y=Y_f, variant=variant)
    want = dst_np.copy()
    oracle.scatter_add_f32(gmap_r, row_lo, _np(Y_f), want, k0)
    dst = torch.from_numpy(dst_np).to(DEV)
    out0 = torch.from_numpy(synth.uniform_f32(81, plan.nnz)).to(DEV)
    out = out0.clone()
    spc.sddmm_spmm_scatter(plan, vals, A, B, dst, k0, kz, out=out, out_mode=out_mode,
                           variant=variant)
    np.testing.assert_array_equal(_bits(_np(dst)), _bits(want), err_msg=f"slab {tag}")
    want_out = out_f if out_mode == spc.OVERWRITE else out0 + out_f
    assert torch.equal(out.view(torch.int32), want_out.view(torch.int32)), f"out {tag}"


def _row_pattern(lengths, ncols, seed, row_lo=0):
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for r, L in enumerate(lengths):
        rows.append(np.full(L, r + row_lo, np.int64))
        cols.append(np.sort(rng.choice(ncols, size=L, replace=False)).astype(np.int64))
    return np.concatenate(rows), np.concatenate(cols)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_scatter_fused_variants(dt):
    spc = _spc()
    p = synth.small_rmat(13, 8, 64, 82, row_range=(1 << 12, 1 << 13), col_range=(0, 1 << 12))
    kz, k0 = 32, 32
    ref = oracle.relabel(p.rows, p.cols, p.row_range, p.col_range)
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range)
    tdt = torch.float32 if dt == "f32" else torch.bfloat16
    A = spc.gather(plan, spc.ROWS, torch.from_numpy(p.A_src).to(DEV), k0, kz, tdt)
    B = spc.gather(plan, spc.COLS, torch.from_numpy(p.B_src).to(DEV), k0, kz, tdt)
    vals = torch.from_numpy(p.vals[ref["perm"]]).to(DEV)
    dst0 = synth.dense_f32(83, 0, p.row_range[1] - p.row_range[0], 96)   # ld 96 > k0 + kz
    for v in (-1, (3, 2), (2, 3, 1), (3, 0, 0, 1), (2, 2, 0, 1), (1, 3)):
        vv = v if isinstance(v, int) else spc.variant(*v)
        for mode in (spc.OVERWRITE, spc.ACCUMULATE):
            _say(f"scatter-fused {dt} variant={v} out_mode={mode} nnz={plan.nnz}")
            _check(spc, plan, ref["gmap_r"], p.row_range[0], vals, A, B, dst0, k0, kz, vv, mode,
                   f"{dt} v={v} mode={mode}")


def test_scatter_fused_long_rows_and_scalar_shape():
    """Rows of 20,000 and 70,000 entries split over many work items (their sums
    finish in the carry fix-up, which then adds them into the slab); a column
    offset k0 = 3 puts the rows off 16-byte alignment (the scalar shape)."""
    spc = _spc()
    lengths = [1, 2, 20000, 3, 70000, 5, 1, 64, 65]
    rows, cols = _row_pattern(lengths, 100_000, 84, row_lo=50)
    rr, cr = (40, 40 + 2 * len(lengths) + 20), (0, 100_000)
    kz = 32
    vals_c = synth.uniform_f32(85, rows.size)
    A_src = synth.dense_f32(86, 0, rr[1] - rr[0], 48)
    B_src = synth.dense_f32(87, 0, cr[1] - cr[0], 48)
    ref = oracle.relabel(rows, cols, rr, cr)
    plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               rr, cr)
    vals = torch.from_numpy(vals_c[ref["perm"]]).to(DEV)
    for k0, variants in ((8, (-1, (3, 0), (2, 1), (3, 0, 0, 1))), (3, (-1, (3, 0, 0, 1)))):
        A = spc.gather(plan, spc.ROWS, torch.from_numpy(A_src).to(DEV), k0, kz)
        B = spc.gather(plan, spc.COLS, torch.from_numpy(B_src).to(DEV), k0, kz)
        dst0 = synth.dense_f32(88, 0, rr[1] - rr[0], 48)
        for v in variants:
            vv = v if isinstance(v, int) else spc.variant(*v)
            _say(f"scatter-fused long rows k0={k0} variant={v}")
            _check(spc, plan, ref["gmap_r"], rr[0], vals, A, B, dst0, k0, kz, vv, spc.OVERWRITE,
                   f"long rows k0={k0} v={v}")


def test_scatter_fused_owner_grouped_rows_and_errors():
    spc = _spc()
    p = synth.small_rmat(12, 8, 32, 89, row_range=(1 << 11, 1 << 12), col_range=(0, 1 << 11))
    rr = p.row_range
    keys = (synth.draws_u64(90, rr[1] - rr[0]) % np.uint64(5)).astype(np.int32)
    ref = oracle.relabel(p.rows, p.cols, rr, p.col_range, group_r=keys, ngroups_r=5)
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               rr, p.col_range, group_r=torch.from_numpy(keys).to(DEV),
                               ngroups_r=5)
    np.testing.assert_array_equal(_np(plan.maps()["gmap_r"]), ref["gmap_r"])
    kz, k0 = 16, 16
    A = spc.gather(plan, spc.ROWS, torch.from_numpy(p.A_src).to(DEV), k0, kz)
    B = spc.gather(plan, spc.COLS, torch.from_numpy(p.B_src).to(DEV), k0, kz)
    vals = torch.from_numpy(p.vals[ref["perm"]]).to(DEV)
    dst0 = synth.dense_f32(91, 0, rr[1] - rr[0], 32)
    _check(spc, plan, ref["gmap_r"], rr[0], vals, A, B, dst0, k0, kz, -1, spc.OVERWRITE, "grouped")
    dst = torch.zeros((rr[1] - rr[0], 32), device=DEV)
    with pytest.raises(ValueError):   # k0 + kz beyond the slab's row: the binding sees it
        spc.sddmm_spmm_scatter(plan, vals, A, B, dst, 20, kz)
    out = torch.empty(plan.nnz, device=DEV)
    buf = torch.empty(spc.spmm_buffer_size(plan, 0, kz), dtype=torch.uint8, device=DEV)
    st = spc.lib().spc3d_sddmm_spmm_scatter(   # and the C entry point refuses it on its own
        plan.handle, vals.data_ptr(), A.data_ptr(), B.data_ptr(), spc.F32, kz, out.data_ptr(),
        spc.OVERWRITE, dst.data_ptr(), dst.stride(0), 20, -1, buf.data_ptr(), buf.numel(),
        torch.cuda.current_stream().cuda_stream)
    assert st == spc.ERR_INVALID_ARG
    with pytest.raises(spc.Spc3dError) as e:
        spc.sddmm_spmm_scatter(plan, vals, A, B, dst, k0, kz, out_mode=7)
    assert e.value.status == spc.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert not bool(dst.any())   # refused calls launch nothing
