"""The hot path under HIP graph capture: the whole step (gather A, gather B,
SDDMM+SpMM fused or separate, scatter-reduce) captured once and replayed
several times, with eager work and synchronizations between the replays;
every replay must equal the eager step bit for bit (the same kernels on the
same inputs).  The library allocates nothing and records no memset in a hot
call, so its launches are all a graph needs."""
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


@pytest.mark.parametrize("form,dtype", [("fused", "f32"), ("separate", "f32"), ("fused", "bf16"),
                                        ("folded", "f32"), ("static", "f32")])
def test_step_graph_replays_equal_eager(form, dtype):
    """form: the fused pass then the scatter-reduce; separate kernels; the
    scatter-reduce folded into the pass (spc3d_sddmm_spmm_scatter); the fused
    pass on the library's static scratch (spc3d_sddmm_spmm_static, the entry
    point meant for callers that capture graphs and cannot allocate)."""
    from paper_2404_19638_amd import spc3d as spc
    p = synth.small_rmat(13, 16, 128, 31, row_range=(1 << 12, 3 << 12), col_range=(0, 1 << 13))
    _say(f"graph form={form} dtype={dtype} nnz={p.nnz}")
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range)
    R, C, nnz, kz, k0 = plan.R, plan.C, plan.nnz, 32, 64
    vals = spc.permute_values(plan, spc.CALLER_TO_SLOT, torch.from_numpy(p.vals).to(DEV))
    A_src = torch.from_numpy(p.A_src).to(DEV)
    B_src = torch.from_numpy(p.B_src).to(DEV)
    Y0 = torch.rand(A_src.shape, generator=torch.Generator().manual_seed(5)).to(DEV)
    pdt = torch.float32 if dtype == "f32" else torch.bfloat16
    A = torch.empty((R, kz), dtype=pdt, device=DEV)
    B = torch.empty((C, kz), dtype=pdt, device=DEV)
    out = torch.empty(nnz, device=DEV)
    Y = torch.empty((R, kz), device=DEV)
    Yd = Y0.clone()
    buf = torch.empty(spc.spmm_buffer_size(plan, 0, kz, -1), dtype=torch.uint8, device=DEV)

    def step():
        spc.gather(plan, spc.ROWS, A_src, k0, kz, packed_dtype=pdt, out=A)
        spc.gather(plan, spc.COLS, B_src, k0, kz, packed_dtype=pdt, out=B)
        if form == "folded":
            spc.sddmm_spmm_scatter(plan, vals, A, B, Yd, k0, kz, out=out, buf=buf)
            return
        if form == "fused":
            spc.sddmm_spmm(plan, vals, A, B, kz, out=out, Y=Y, buf=buf)
        elif form == "static":
            spc.sddmm_spmm_static(plan, vals, A, B, kz, out=out, Y=Y)
        else:
            spc.sddmm(plan, vals, A, B, kz, out=out)
            spc.spmm(plan, vals, B, 0, kz, out=Y, buf=buf)
        spc.scatter_reduce(plan, spc.ROWS, Y, Yd, k0)

    step()   # eager reference (and warm-up outside the capture)
    torch.cuda.synchronize()
    want = [t.clone() for t in (A, B, out, Y, Yd)]

    g = torch.cuda.CUDAGraph()
    Yd.copy_(Y0)
    for t in (A, B, out, Y):
        t.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for rep in range(3):
        Yd.copy_(Y0)
        for t in (A, B, out, Y):
            t.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for name, got, ref in zip(("A_loc", "B_loc", "out", "Y_loc", "Y_dst"), (A, B, out, Y, Yd),
                                  want):
            if form == "folded" and name == "Y_loc":
                continue   # the folded pass writes no packed Y
            assert torch.equal(got.view(torch.int16 if got.dtype == torch.bfloat16 else torch.int32),
                               ref.view(torch.int16 if ref.dtype == torch.bfloat16 else torch.int32)), \
                (rep, name)
        # eager work between replays: an unrelated library call and torch ops
        spc.sddmm(plan, None, A, B, kz, out=torch.empty(nnz, device=DEV))
        (A_src[:1000] * 2).sum().item()
        torch.cuda.synchronize()
    # back-to-back replays accumulate into the owner's slab like eager steps
    Yd.copy_(Y0)
    g.replay()
    g.replay()
    torch.cuda.synchronize()
    Y2 = Yd.clone()
    Yd.copy_(Y0)
    step()
    step()
    torch.cuda.synchronize()
    assert torch.equal(Y2.view(torch.int32), Yd.view(torch.int32))
    del g


@pytest.mark.parametrize("fused", [False, True])
def test_attention_training_step_graph_replays_equal_eager(fused):
    """Forward and hand-written backward of the graph-attention layer (three
    kernels, or the fused one-pass forward) captured in one HIP graph: each
    replay, with eager work between replays, gives the eager step's output and
    gradients bit for bit.  The backward is seeded with an explicit output
    gradient, so no reduction kernel of the loss enters the graph."""
    from paper_2404_19638_amd import spc3d as spc
    from paper_2404_19638_amd import autograd as ag
    p = synth.small_rmat(11, 8, 32, 99, row_range=(1 << 10, 1 << 11), col_range=(0, 1 << 10))
    plan = spc.plan_create_coo(torch.from_numpy(p.rows).to(DEV), torch.from_numpy(p.cols).to(DEV),
                               p.row_range, p.col_range, spc.BUILD_CSC)
    _say(f"attention graph fused={fused} nnz={plan.nnz}")
    g = torch.Generator().manual_seed(7)
    Q = torch.randn((plan.R, 32), generator=g).to(DEV).requires_grad_()
    Kf = torch.randn((plan.C, 32), generator=g).to(DEV).requires_grad_()
    V = torch.randn((plan.C, 32), generator=g).to(DEV).requires_grad_()
    G = torch.randn((plan.R, 32), generator=g).to(DEV)

    def step():
        for t in (Q, Kf, V):
            t.grad = None
        out = ag.gnn_attention(plan, Q, Kf, V, fused=fused)
        torch.autograd.backward(out, G)
        return out

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # warm-up (buffers, autograd state) off the capture
        for _ in range(2):
            out = step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    want = [out.detach().clone()] + [t.grad.clone() for t in (Q, Kf, V)]
    del out   # drop the warm-up's autograd graph before the capture builds its own

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out_s = step()
    grads_s = [t.grad for t in (Q, Kf, V)]
    torch.cuda.synchronize()
    for rep in range(3):
        for t in [out_s] + grads_s:
            t.detach().fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        for name, got, ref in zip(("out", "dQ", "dKf", "dV"), [out_s] + grads_s, want):
            assert torch.equal(got.detach().view(torch.int32), ref.view(torch.int32)), (rep, name)
        spc.sddmm(plan, None, Q.detach(), Kf.detach())   # eager work between replays
        torch.cuda.synchronize()
    del graph
