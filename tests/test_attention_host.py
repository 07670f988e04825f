"""Host logic of gnn_attention's automatic forward choice (no GPU needed:
the choice reads only shapes, dtypes, alignment, the grad mode and the
plan's entry count)."""
import types

import pytest

torch = pytest.importorskip("torch")
from paper_2404_19638_amd import autograd as ag   # noqa: E402


def _t(n, k, dt, grad=False):
    t = torch.zeros((n, k), dtype=dt)
    return t.requires_grad_() if grad else t


def test_auto_choice_takes_the_one_pass_forward_only_for_inference():
    small = types.SimpleNamespace(nnz=1000)
    big = types.SimpleNamespace(nnz=ag.AUTO_FUSED_F32_MAX_NNZ + 1)
    bf, f32 = torch.bfloat16, torch.float32
    qkv = lambda dt, k=64, grad=False: (_t(8, k, dt, grad), _t(8, k, dt), _t(8, k, dt))  # noqa: E731
    # inference: bfloat16 at any size, FP32 up to the limit
    assert ag._auto_fused(big, *qkv(bf))
    assert ag._auto_fused(small, *qkv(f32))
    assert ag._auto_fused(types.SimpleNamespace(nnz=ag.AUTO_FUSED_F32_MAX_NNZ), *qkv(f32))
    assert not ag._auto_fused(big, *qkv(f32))
    # a gradient to record: the three kernels, unless grad mode is off
    assert not ag._auto_fused(small, *qkv(bf, grad=True))
    with torch.no_grad():
        assert ag._auto_fused(small, *qkv(bf, grad=True))
    # widths the one-pass kernel does not cover, mixed types, unaligned views
    assert not ag._auto_fused(small, *qkv(f32, k=8))
    assert not ag._auto_fused(small, *qkv(bf, k=12))
    assert not ag._auto_fused(small, _t(8, 64, bf), _t(8, 64, f32), _t(8, 64, bf))
    q, k, v = qkv(f32)
    wide = torch.zeros((8, 65), dtype=f32)
    assert not ag._auto_fused(small, wide[:, 1:], k, v)
    assert not ag._auto_fused(small, q.to(torch.float64), k.to(torch.float64),
                              v.to(torch.float64))
