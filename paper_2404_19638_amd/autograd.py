"""Hand-written backward passes of the local hot path (torch.autograd).

Every forward and backward step is a call into libspc3d; PyTorch only holds
the tensors and records the graph.  The gradients follow from the two
definitions (Eq. (1) and Eq. (2) of the paper) by the chain rule, and each is
itself one of the library's kernels:

  SDDMM   c_p = s_p <a_i, b_j>      (i = row, j = column of slot p)
          dA  = SpMM(S o dC, B)            dB  = SpMM^T(S o dC, A)
          ds  = SDDMM(dC, A, B)            (sampling values dC_p)
  SpMM    y_i = sum_p s_p b_j
          dB  = SpMM^T(S, dY)              ds  = SDDMM(pattern, dY, B)
  softmax alpha = rowsoftmax(e)            de  = alpha o (dalpha - rowsum(alpha o dalpha))
  gather  packed = src[gmap]               dsrc = scatter-add(dpacked)
  scatter dst += packed[...]               dpacked = gather(ddst)

Gradients with respect to A and B of the transposed SpMM need the plan's
column-major view (SPC3D_BUILD_CSC).

Dense operands may be bfloat16 (the library accumulates in FP32): outputs
are FP32, the upstream gradient of a product with bfloat16 operands is
rounded to bfloat16 before it enters the backward kernels (half the bytes
per gathered row), and each returned gradient has its input's type.
"""
from __future__ import annotations

import torch

from . import spc3d as spc


def _needs(ctx, i):
    return ctx.needs_input_grad[i]


def _spmm_t(plan, vals, X):
    """Transposed SpMM (sum over each column's entries).  Values are first
    permuted to column-major order so the kernel reads them as one stream
    rather than one random load per entry through the slot map (the same
    results, bit for bit)."""
    if vals is None:
        return spc.spmm(plan, None, X, transpose=1)
    vt = spc.permute_values(plan, spc.SLOT_TO_COLUMN, vals)
    return spc.spmm(plan, vt, X, transpose=2)


def _as(grad, like):
    """A gradient (FP32 from the library) in the type of its input: with
    bfloat16 operands the products still accumulate in FP32 and only the
    returned gradient is rounded."""
    return grad if grad.dtype == like.dtype else grad.to(like.dtype)


class SDDMMFn(torch.autograd.Function):
    """out = SDDMM(plan, vals, A, B); vals None means pattern-only (s == 1)."""

    @staticmethod
    def forward(ctx, plan, vals, A, B):
        ctx.plan = plan
        # the kernels take packed operands: a sliced input (e.g. a column block
        # of a wider tensor) is copied once and the copy serves both passes
        vals = None if vals is None else vals.contiguous()
        A, B = A.contiguous(), B.contiguous()
        ctx.save_for_backward(vals if vals is not None else torch.empty(0), A, B)
        ctx.has_vals = vals is not None
        return spc.sddmm(plan, vals, A, B)

    @staticmethod
    def backward(ctx, dout):
        plan = ctx.plan
        vals, A, B = ctx.saved_tensors
        dout = dout.contiguous()
        w = spc.mul_values(plan, dout, vals) if ctx.has_vals else dout
        dvals = dA = dB = None
        if ctx.has_vals and _needs(ctx, 1):
            dvals = spc.sddmm(plan, dout, A, B)
        if _needs(ctx, 2):
            dA = _as(spc.spmm(plan, w, B, transpose=0), A)
        if _needs(ctx, 3):
            dB = _as(_spmm_t(plan, w, A), B)
        return None, dvals, dA, dB


class SpMMFn(torch.autograd.Function):
    """Y = SpMM(plan, vals, X) over rows (transpose 0) or columns (transpose 1)."""

    @staticmethod
    def forward(ctx, plan, vals, X, transpose=0):
        ctx.plan = plan
        ctx.transpose = transpose
        ctx.has_vals = vals is not None
        vals = None if vals is None else vals.contiguous()
        X = X.contiguous()
        ctx.save_for_backward(vals if vals is not None else torch.empty(0), X)
        return spc.spmm(plan, vals, X, transpose=transpose)

    @staticmethod
    def backward(ctx, dY):
        plan = ctx.plan
        vals, X = ctx.saved_tensors
        dY = dY.contiguous()
        dvals = dX = None
        dYx = dY.to(X.dtype)   # the upstream gradient in X's type (bfloat16 rows gather half the bytes)
        if ctx.has_vals and _needs(ctx, 1):
            # d y_i / d s_p = x_j: one dot per slot
            if ctx.transpose == 0:
                dvals = spc.sddmm(plan, None, dYx, X)
            else:
                dvals = spc.sddmm(plan, None, X, dYx)
        if _needs(ctx, 2):
            v = vals if ctx.has_vals else None
            if ctx.transpose == 0:
                dX = _as(_spmm_t(plan, v, dYx), X)
            else:
                dX = _as(spc.spmm(plan, v, dYx, transpose=0), X)
        return None, dvals, dX, None


class RowSoftmaxFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, plan, e):
        alpha = spc.row_softmax(plan, e.contiguous())
        ctx.plan = plan
        ctx.save_for_backward(alpha)
        return alpha

    @staticmethod
    def backward(ctx, dalpha):
        (alpha,) = ctx.saved_tensors
        return None, spc.row_softmax_bwd(ctx.plan, alpha, dalpha.contiguous())


class GatherFn(torch.autograd.Function):
    """packed = rows gmap[l] - lo of src, columns [k0, k0+kz) (FP32)."""

    @staticmethod
    def forward(ctx, plan, axis, src, k0, kz):
        ctx.plan, ctx.axis, ctx.k0, ctx.shape = plan, axis, k0, src.shape
        return spc.gather(plan, axis, src, k0, kz)

    @staticmethod
    def backward(ctx, dpacked):
        dsrc = torch.zeros(ctx.shape, dtype=torch.float32, device=dpacked.device)
        spc.scatter_reduce(ctx.plan, ctx.axis, dpacked.contiguous(), dsrc, ctx.k0)
        return None, None, dsrc, None, None


class ScatterReduceFn(torch.autograd.Function):
    """Returns dst + (packed rows added at gmap rows, columns k0..k0+kz)."""

    @staticmethod
    def forward(ctx, plan, axis, packed, dst, k0):
        ctx.plan, ctx.axis, ctx.k0, ctx.kz = plan, axis, k0, packed.shape[1]
        out = dst.clone()
        spc.scatter_reduce(plan, axis, packed.contiguous(), out, k0)
        return out

    @staticmethod
    def backward(ctx, dout):
        dout = dout.contiguous()
        dpacked = spc.gather(ctx.plan, ctx.axis, dout, ctx.k0, ctx.kz)
        return None, None, dpacked, dout, None


class FusedAttentionFn(torch.autograd.Function):
    """out = rowsoftmax(SDDMM(pattern, Q, Kf)) . V in one fused pass
    (spc3d_attention_fwd).  The backward recomputes the scores with one SDDMM,
    rebuilds alpha from the stored row (max, sum) pairs, and then runs the
    chain of the unfused layer: dalpha = SDDMM(dout, V), de = softmax
    backward, dQ = SpMM(de, Kf), dKf = SpMM^T(de, Q), dV = SpMM^T(alpha, dout)."""

    @staticmethod
    def forward(ctx, plan, Q, Kf, V):
        Q, Kf, V = Q.contiguous(), Kf.contiguous(), V.contiguous()
        out, stats = spc.attention_fwd(plan, Q, Kf, V)
        ctx.plan = plan
        ctx.save_for_backward(Q, Kf, V, stats)
        return out

    @staticmethod
    def backward(ctx, dout):
        plan = ctx.plan
        Q, Kf, V, stats = ctx.saved_tensors
        dout = dout.contiguous()
        e = spc.sddmm(plan, None, Q, Kf)
        alpha = spc.row_softmax_apply(plan, e, stats, out=e)
        dout = dout.to(V.dtype)   # the upstream gradient in the operands' type
        dalpha = spc.sddmm(plan, None, dout, V)
        de = spc.row_softmax_bwd(plan, alpha, dalpha, out=dalpha)
        dQ = dK = dV = None
        if _needs(ctx, 1):
            dQ = _as(spc.spmm(plan, de, Kf, transpose=0), Q)
        if _needs(ctx, 2):
            dK = _as(_spmm_t(plan, de, Q), Kf)
        if _needs(ctx, 3):
            dV = _as(_spmm_t(plan, alpha, dout), V)
        return None, dQ, dK, dV


def sddmm(plan, vals, A, B):
    return SDDMMFn.apply(plan, vals, A, B)


def spmm(plan, vals, X, transpose=0):
    return SpMMFn.apply(plan, vals, X, transpose)


def row_softmax(plan, e):
    return RowSoftmaxFn.apply(plan, e)


def gather(plan, axis, src, k0, kz):
    return GatherFn.apply(plan, axis, src, k0, kz)


def scatter_reduce(plan, axis, packed, dst, k0):
    return ScatterReduceFn.apply(plan, axis, packed, dst, k0)


def _need_fused(Q, Kf, V):
    dt = spc.BF16 if Q.dtype == torch.bfloat16 else spc.F32
    if not spc.attention_supported(Q.shape[1], dt):
        raise ValueError(f"the fused attention pass does not cover K={Q.shape[1]}")
    if not all(t.data_ptr() % 16 == 0 for t in (Q, Kf, V)):
        raise ValueError("the fused attention pass needs 16-byte aligned Q, Kf and V")


# Largest FP32 block (stored entries) on which the automatic choice takes the
# one-pass forward: it measured faster at 1.8M entries (R-MAT 2^16, K = 64) and
# slower from 7.6M entries (2^18) on, where the Kf and V rows it keeps live
# together outgrow the Infinity Cache.  With bfloat16 operands it measured
# faster at every size up to 31.4M entries (2^20).
AUTO_FUSED_F32_MAX_NNZ = 1 << 21


def _auto_fused(plan, Q, Kf, V):
    """The forward gnn_attention takes when the caller leaves it open: the
    one-pass kernel for inference (no gradient is recorded) where it measured
    faster, the three kernels otherwise (the fused backward recomputes the
    scores, and the fused forward loses in FP32 on large blocks)."""
    if torch.is_grad_enabled() and any(t.requires_grad for t in (Q, Kf, V)):
        return False
    if not (Q.dtype == Kf.dtype == V.dtype) or Q.dtype not in (torch.float32, torch.bfloat16):
        return False
    dt = spc.BF16 if Q.dtype == torch.bfloat16 else spc.F32
    if not spc.attention_supported(Q.shape[1], dt):
        return False
    if not all(t.is_contiguous() and t.data_ptr() % 16 == 0 for t in (Q, Kf, V)):
        return False
    return dt == spc.BF16 or plan.nnz <= AUTO_FUSED_F32_MAX_NNZ


def gnn_attention(plan, Q, Kf, V, fused: bool | None = None):
    """Masked attention over the block's pattern: SDDMM edge scores (s == 1),
    row softmax over each row's stored entries, SpMM aggregation of V.

    Q is [R, K] (local rows), Kf and V are [C, K] (local columns); returns [R, K].
    fused=True runs the forward as one pass (spc3d_attention_fwd; K must be
    covered by it, see spc.attention_supported) and recomputes the scores in
    the backward; fused=False runs the three separate kernels.  Left as None,
    the one-pass forward is taken for inference (no gradient recorded) with
    bfloat16 operands, or FP32 operands on blocks of up to
    AUTO_FUSED_F32_MAX_NNZ entries, and the three kernels otherwise: the
    layer is bound by the gathers of Kf and V rows, which the fused pass
    keeps live together, so in FP32 it measured slower on large blocks.
    """
    if fused is None:
        fused = _auto_fused(plan, Q, Kf, V)
    if fused:
        _need_fused(Q, Kf, V)
        return FusedAttentionFn.apply(plan, Q, Kf, V)
    e = sddmm(plan, None, Q, Kf)
    alpha = row_softmax(plan, e)
    return spmm(plan, alpha, V, 0)
