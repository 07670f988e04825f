"""The library's default shapes (variant -1) in every size class they
distinguish, each output compared element by element with the FP64 oracle.

The default picks the lanes per entry, the work-item size and the SpMM
family from the operand type, the row width and the block's entry count,
with thresholds at 2^18, 2^20 and 2^21 entries.  Blocks just inside each class
(uniform positions, about 8 entries per row) run the fused SDDMM+SpMM at
kz = 16, 32, 64 and 128 with FP32 and bfloat16 operands, SDDMM and SpMM on
their own where their own defaults differ, and the pass with the
scatter-reduce folded in.

Bars: |x - x*| <= 1e-5 M, M the oracle's magnitude sum, for FP32 operands and
for bfloat16 operands against the oracle on the same rounded inputs; the
folded slab bit for bit against the oracle's FP32 addition of the plain
pass's rows."""
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
# one block per size class of the default rule: [0, 2^18), [2^18, 2^20),
# [2^20, 2^21), [2^21, ...)
CLASSES = {"below 2^18": (1 << 17) + 7, "2^18 to 2^20": (1 << 19) + 3,
           "2^20 to 2^21": 1_400_001, "from 2^21": 2_300_003}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _spc():
    from paper_2404_19638_amd import spc3d
    return spc3d


def _np(t):
    return t.detach().float().cpu().numpy()


_BLOCKS = {}


def _block(name):
    """Plan, oracle localization and caller-order entries of a uniform block
    with the class's entry count (kept for the module: built once)."""
    if name not in _BLOCKS:
        spc = _spc()
        nnz = CLASSES[name]
        n = max(1024, nnz // 8)
        rows, cols = synth.uniform_block(n, n, nnz, 300 + list(CLASSES).index(name))
        rr = cr = (0, n)
        plan = spc.plan_create_coo(torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                                   rr, cr)
        ref = oracle.relabel(rows, cols, rr, cr)
        assert plan.nnz == nnz
        vals = synth.uniform_f32(401, nnz)
        _BLOCKS[name] = (plan, ref, rows, cols, n, vals)
    return _BLOCKS[name]


def _operands(n, kz, bf16, seed):
    A = synth.dense_f32(seed, 0, n, kz)
    B = synth.dense_f32(seed + 1, 0, n, kz)
    if bf16:
        A = oracle.bf16_to_f32(oracle.bf16_rne(A))
        B = oracle.bf16_to_f32(oracle.bf16_rne(B))
    return A, B


def _packed(x, gmap, bf16):
    t = torch.from_numpy(np.ascontiguousarray(x[gmap])).to(DEV)
    return t.bfloat16() if bf16 else t   # exact: the values are already bfloat16


@pytest.mark.parametrize("name", list(CLASSES))
@pytest.mark.parametrize("bf16", [False, True], ids=["f32", "bf16"])
def test_fused_default_shape_in_every_size_class(name, bf16):
    spc = _spc()
    plan, ref, rows, cols, n, vals = _block(name)
    v_slot = torch.from_numpy(vals[ref["perm"]]).to(DEV)
    for kz in (16, 32, 64, 128):
        _say(f"default fused pass: {name} nnz={plan.nnz} kz={kz} {'bf16' if bf16 else 'f32'}")
        A, B = _operands(n, kz, bf16, 500 + kz)
        out, Y = spc.sddmm_spmm(plan, v_slot, _packed(A, ref["gmap_r"], bf16),
                                _packed(B, ref["gmap_c"], bf16), kz)
        o, mo = oracle.sddmm(rows, cols, 0, 0, vals, A, B, 0, kz)
        assert_within_mag(_np(out), o[ref["perm"]], mo[ref["perm"]], 1e-5,
                          f"sddmm {name} kz={kz}")
        y, my = oracle.spmm(rows, cols, 0, 0, ref["lmap_r"], ref["R"], vals, B, 0, kz)
        assert_within_mag(_np(Y), y, my, 1e-5, f"spmm {name} kz={kz}")


@pytest.mark.parametrize("name", list(CLASSES))
def test_separate_default_shapes_where_they_differ(name):
    """FP32 SDDMM at kz = 64 and 128 (8 lanes per entry below 2^20 entries),
    FP32 and bfloat16 SpMM at kz = 16 (the windowed family from 2^18 to 2^20
    entries for FP32)."""
    spc = _spc()
    plan, ref, rows, cols, n, vals = _block(name)
    v_slot = torch.from_numpy(vals[ref["perm"]]).to(DEV)
    for kz in (64, 128):
        _say(f"default SDDMM: {name} kz={kz}")
        A, B = _operands(n, kz, False, 600 + kz)
        out = spc.sddmm(plan, v_slot, _packed(A, ref["gmap_r"], False),
                        _packed(B, ref["gmap_c"], False), kz)
        o, mo = oracle.sddmm(rows, cols, 0, 0, vals, A, B, 0, kz)
        assert_within_mag(_np(out), o[ref["perm"]], mo[ref["perm"]], 1e-5, f"sddmm {name}")
    for bf16 in (False, True):
        _say(f"default SpMM: {name} kz=16 {'bf16' if bf16 else 'f32'}")
        _, B = _operands(n, 16, bf16, 700)
        Y = spc.spmm(plan, v_slot, _packed(B, ref["gmap_c"], bf16), 0, 16)
        y, my = oracle.spmm(rows, cols, 0, 0, ref["lmap_r"], ref["R"], vals, B, 0, 16)
        assert_within_mag(_np(Y), y, my, 1e-5, f"spmm {name}")


@pytest.mark.parametrize("name", ["2^18 to 2^20", "from 2^21"])
@pytest.mark.parametrize("kz", [16, 128])
def test_folded_pass_default_shape(name, kz):
    """The pass with the scatter-reduce folded in, in the default shapes that
    the refinements introduced (windowed for narrow rows from 2^18 entries;
    half the lanes and 256-slot work items for bfloat16 at kz = 128 from 2^21):
    the slab bit for bit as the oracle's FP32 addition of the plain pass's
    rows."""
    spc = _spc()
    plan, ref, rows, cols, n, vals = _block(name)
    v_slot = torch.from_numpy(vals[ref["perm"]]).to(DEV)
    A, B = _operands(n, kz, True, 800 + kz)
    Ad, Bd = _packed(A, ref["gmap_r"], True), _packed(B, ref["gmap_c"], True)
    _, Y = spc.sddmm_spmm(plan, v_slot, Ad, Bd, kz)
    k0, K = 16, kz + 32
    dst0 = synth.dense_f32(901, 0, n, K)
    want = dst0.copy()
    oracle.scatter_add_f32(ref["gmap_r"], 0, _np(Y), want, k0)
    dst = torch.from_numpy(dst0).to(DEV)
    _say(f"default folded pass: {name} kz={kz} bf16")
    spc.sddmm_spmm_scatter(plan, v_slot, Ad, Bd, dst, k0, kz)
    np.testing.assert_array_equal(_np(dst).view(np.uint32), want.view(np.uint32))
