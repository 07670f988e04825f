"""spc3d_plan_check and the SPC3D_DEBUG_BOUNDS mode.

Valid plans (R-MAT with the column-major arrays, a ragged uniform block, an
owner-grouped plan, a plan from CSR input, a block with one entry, an empty
block) pass the check.  A plan with one local id overwritten from the host
(through the device views of spc3d_plan_maps) fails it with OUT_OF_RANGE,
naming the invariant and the index; every such damage is undone before the
next, and the check only reads the plan's arrays, so no kernel runs on a
damaged id.  In a child process with SPC3D_DEBUG_BOUNDS=1, an SDDMM on a
damaged plan returns the check's error before launching, and after the
damage is undone the same call gives the result of the unchecked library."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2404_19638_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():   # pragma: no cover
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

DEV = "cuda:0"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _plan(spc, rows, cols, rr, cr, flags=0, **kw):
    return spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                               rr, cr, flags, **kw)


def test_valid_plans_pass():
    spc = _spc()
    p = synth.small_rmat(12, 8, 32, 91, row_range=(1 << 11, 1 << 12), col_range=(0, 1 << 11))
    plans = [("rmat csc", _plan(spc, p.rows, p.cols, p.row_range, p.col_range, spc.BUILD_CSC))]
    r, c = synth.uniform_block(700, 900, 3001, 92)
    plans.append(("uniform ragged", _plan(spc, r, c, (0, 700), (0, 900), spc.BUILD_CSC)))
    keys = (np.arange(p.row_range[1] - p.row_range[0]) % 5).astype(np.int32)
    plans.append(("grouped", _plan(spc, p.rows, p.cols, p.row_range, p.col_range,
                                   group_r=torch.from_numpy(keys).to(DEV), ngroups_r=5)))
    order = np.lexsort((p.cols, p.rows))
    rows_s, cols_s = p.rows[order], p.cols[order]
    nr = p.row_range[1] - p.row_range[0]
    rowptr = np.searchsorted(rows_s, np.arange(p.row_range[0], p.row_range[1] + 1)).astype(np.int64)
    plans.append(("csr input", spc.plan_create_csr(torch.from_numpy(rowptr).to(DEV),
                                                   torch.from_numpy(cols_s).to(DEV),
                                                   p.row_range, p.col_range, spc.BUILD_CSC)))
    assert nr + 1 == rowptr.size
    one = np.array([5], np.int64)
    plans.append(("one entry", _plan(spc, one, one, (0, 8), (0, 8), spc.BUILD_CSC)))
    empty = np.zeros(0, np.int64)
    plans.append(("empty", _plan(spc, empty, empty, (0, 8), (0, 8), spc.BUILD_CSC)))
    for name, plan in plans:
        _say(f"plan check, valid plan: {name} nnz={plan.nnz}")
        spc.plan_check(plan)


DAMAGES = [
    # (array, index picker, new value, words the error must contain)
    ("colidx", lambda pl, a: pl.nnz // 2, lambda pl: pl.C + 5, "colidx outside [0, C)"),
    ("colidx", lambda pl, a: 0, lambda pl: -1, "colidx outside [0, C)"),
    ("rowptr", lambda pl, a: pl.R // 2, lambda pl: 0, "rowptr"),
    ("perm", lambda pl, a: pl.nnz - 1, lambda pl: pl.nnz, "perm outside [0, nnz)"),
    ("gmap_r", lambda pl, a: pl.R - 1, lambda pl: pl.row_range[1], "gmap_r"),
    ("gmap_c", lambda pl, a: 1, lambda pl: pl.col_range[0] - 1, "gmap_c"),
    ("rowidx_t", lambda pl, a: 7, lambda pl: pl.R, "rowidx_t outside [0, R)"),
    ("slot_t", lambda pl, a: pl.nnz // 3, lambda pl: -3, "slot_t outside [0, nnz)"),
    ("colptr", lambda pl, a: pl.C, lambda pl: pl.nnz + 1, "colptr"),
]


@pytest.mark.parametrize("array,pick,value,words", DAMAGES,
                         ids=[f"{d[0]}-{i}" for i, d in enumerate(DAMAGES)])
def test_damaged_plan_fails_the_check(array, pick, value, words):
    spc = _spc()
    p = synth.small_rmat(12, 8, 32, 93, row_range=(1 << 11, 1 << 12), col_range=(0, 1 << 11))
    plan = _plan(spc, p.rows, p.cols, p.row_range, p.col_range, spc.BUILD_CSC)
    spc.plan_check(plan)
    a = plan.maps()[array]
    i = pick(plan, a)
    old = a[i].item()
    _say(f"plan check, damaged {array}[{i}]: {old} -> {value(plan)}")
    a[i] = value(plan)
    torch.cuda.synchronize()
    try:
        with pytest.raises(spc.Spc3dError) as ei:
            spc.plan_check(plan)
        assert ei.value.status == spc.ERR_OUT_OF_RANGE
        assert words in str(ei.value), str(ei.value)
    finally:
        a[i] = old
        torch.cuda.synchronize()
    spc.plan_check(plan)


CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2404_19638_amd import spc3d as spc, synth
assert spc.debug_bounds()
dev = "cuda:0"
p = synth.small_rmat(12, 8, 32, 94, row_range=(1 << 11, 1 << 12), col_range=(0, 1 << 11))
plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(dev), torch.from_numpy(p.cols).to(dev),
                           p.row_range, p.col_range)
A = torch.from_numpy(synth.dense_f32(1, 0, plan.R, 32)).to(dev)
B = torch.from_numpy(synth.dense_f32(2, 0, plan.C, 32)).to(dev)
want = torch.from_numpy(np.frombuffer(sys.stdin.buffer.read(), dtype=np.int32).copy())
got = spc.sddmm(plan, None, A, B, 32)
assert torch.equal(got.view(torch.int32).cpu(), want), "checked call differs"
col = plan.maps()["colidx"]
old = col[3].item()
col[3] = plan.C + 100
torch.cuda.synchronize()
try:
    spc.sddmm(plan, None, A, B, 32)
    raise SystemExit("damaged plan accepted")
except spc.Spc3dError as e:
    assert e.status == spc.ERR_OUT_OF_RANGE and "colidx" in str(e), str(e)
col[3] = old
torch.cuda.synchronize()
got = spc.sddmm(plan, None, A, B, 32)
assert torch.equal(got.view(torch.int32).cpu(), want), "after repair"
print("debug bounds child: ok", flush=True)
"""


def test_debug_bounds_mode_refuses_a_damaged_plan_before_launching():
    spc = _spc()
    assert not spc.debug_bounds()
    p = synth.small_rmat(12, 8, 32, 94, row_range=(1 << 11, 1 << 12), col_range=(0, 1 << 11))
    plan = _plan(spc, p.rows, p.cols, p.row_range, p.col_range)
    A = torch.from_numpy(synth.dense_f32(1, 0, plan.R, 32)).to(DEV)
    B = torch.from_numpy(synth.dense_f32(2, 0, plan.C, 32)).to(DEV)
    want = spc.sddmm(plan, None, A, B, 32).view(torch.int32).cpu().numpy().tobytes()
    _say("plan check: debug-bounds child process")
    env = dict(os.environ, SPC3D_DEBUG_BOUNDS="1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], input=want, env=env,
                       capture_output=True, timeout=300)
    out = r.stdout.decode() + r.stderr.decode()
    assert r.returncode == 0 and "debug bounds child: ok" in out, out[-3000:]
