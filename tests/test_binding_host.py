"""Host-side shape checks of the Python binding (CPU only): calls whose
tensors the kernels would read with the wrong shape raise ValueError before
anything reaches the C library."""
import types

import pytest

torch = pytest.importorskip("torch")
from paper_2404_19638_amd import spc3d as spc   # noqa: E402

PLAN = types.SimpleNamespace(R=10, C=12, nnz=30, row_range=(100, 120), col_range=(0, 16),
                             handle=None)


def test_gather_columns_must_lie_inside_src():
    src = torch.zeros((20, 48))
    with pytest.raises(ValueError, match="k0..k0\\+kz"):
        spc.gather(PLAN, spc.ROWS, src, 32, 32)
    with pytest.raises(ValueError, match="k0..k0\\+kz"):
        spc.gather(PLAN, spc.ROWS, src, -1, 8)


def test_packed_operands_must_have_kz_columns():
    A, B = torch.zeros((10, 64)), torch.zeros((12, 64))
    with pytest.raises(ValueError, match="kz columns"):
        spc.sddmm(PLAN, None, A, B, 32)
    with pytest.raises(ValueError, match="kz columns"):
        spc.sddmm_spmm(PLAN, None, A, B, 32)
    with pytest.raises(ValueError, match="kz columns"):
        spc.sddmm_spmm_static(PLAN, None, A, B, 32)
    with pytest.raises(ValueError, match="kz columns"):
        spc.spmm(PLAN, None, torch.zeros((12, 64)), 0, 32)
    A32, B32 = torch.zeros((10, 32)), torch.zeros((12, 32))
    with pytest.raises(ValueError, match="R rows of kz"):
        spc.sddmm_spmm(PLAN, None, A32, B32, 32, Y=torch.zeros((10, 33)))
    with pytest.raises(ValueError, match="n rows of kz"):
        spc.spmm(PLAN, None, B32, 0, 32, out=torch.zeros((10, 31)))


def test_scatter_columns_must_lie_inside_dst():
    dst = torch.zeros((20, 40))
    with pytest.raises(ValueError, match="k0..k0\\+kz"):
        spc.scatter_reduce(PLAN, spc.ROWS, torch.zeros((10, 32)), dst, 16)
    A32, B32 = torch.zeros((10, 32)), torch.zeros((12, 32))
    with pytest.raises(ValueError, match="k0..k0\\+kz"):
        spc.sddmm_spmm_scatter(PLAN, None, A32, B32, dst, 16, 32)
