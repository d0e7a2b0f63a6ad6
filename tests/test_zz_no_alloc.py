"""The no-allocation step (nmf_beta_step_noalloc) through the C ABI, against
the allocating step (nmf_beta_step) on the same inputs.

Both run the same kernels with the same launch plan, so the results must be
bitwise equal; they are also checked against the FP64 oracle with the usual
float32 gates.  Two calls in a row, the second smaller: the fixed per-GPU
scratch array keeps the first call's contents, which the second must not
depend on.  Also: capture into a HIP graph on a context that never reserved
a workspace, an oversized step rejected before any device work, and the
caller's flag word.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import synth
import paper_2106_15214_amd as nb
from gates import check_pair

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
NMF_ERR_WORKSPACE = 5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def noalloc(ctx, V, W, H, beta, mode, obj=None, flags=None, inner_iters=1, stream=None):
    """Direct ctypes call of the C entry point (no binding logic in between)."""
    L = nb.lib()
    o = nb._opts(inner_iters=inner_iters)
    s = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    return L.nmf_beta_step_noalloc(ctx.handle, s, V.shape[0], V.shape[1], W.shape[1], V.data_ptr(), V.stride(0),
                                   W.data_ptr(), W.stride(0), H.data_ptr(), H.stride(0), float(beta),
                                   nb.MODES[mode], ctypes.byref(o), obj.data_ptr() if obj is not None else None,
                                   flags.data_ptr() if flags is not None else None)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_noalloc_matches_step_two_calls_second_smaller(mode, beta):
    ctx = nb.Context(0)
    ref_ctx = nb.Context(0)
    for call, (F, N, K) in enumerate([(700, 900, 40), (150, 333, 17)]):
        p = synth.random_positive(F, N, K, seed=800 + call, zeros=0.1)
        print(f"[noalloc] call {call} F={F} N={N} K={K} beta={beta} mode={mode}", flush=True)
        V = dev(p.V)
        Wa, Ha = dev(p.W), dev(p.H)
        Wb, Hb = dev(p.W), dev(p.H)
        oa = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
        ob = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
        fl = torch.zeros(1, dtype=torch.int32, device=DEV)
        assert noalloc(ctx, V, Wa, Ha, beta, mode, obj=oa, flags=fl) == 0
        nb.step(V, Wb, Hb, beta, mode, objective_out=ob, ctx=ref_ctx)
        torch.cuda.synchronize()
        assert fl.item() == 0 and nb.get_flags(clear=True, ctx=ref_ctx) == 0
        assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb), "no-allocation step differs from nmf_beta_step"
        assert oa.item() == ob.item()
        f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
        V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
        Wr, Hr = f(V64, W64, H64, beta)
        check_pair(Wa.cpu().numpy(), Ha.cpu().numpy(), Wr, Hr, tag=f"noalloc call {call}")
        d0 = O.objective(V64, W64, H64, beta)
        assert abs(oa.item() - d0) <= 1e-6 * abs(d0)
    ctx.close()
    ref_ctx.close()


def test_noalloc_sub_iterations_and_binding():
    ctx = nb.Context(0)
    p = synth.random_positive(257, 300, 20, seed=810, zeros=0.1)
    V = dev(p.V)
    Wa, Ha, Wb, Hb = dev(p.W), dev(p.H), dev(p.W), dev(p.H)
    nb.step_noalloc(V, Wa, Ha, 0.5, "joint", inner_iters=2, ctx=ctx)
    nb.step(V, Wb, Hb, 0.5, "joint", inner_iters=2, ctx=ctx)
    torch.cuda.synchronize()
    assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb)
    ctx.close()


def test_noalloc_under_graph_capture_without_reserve():
    # a fresh context that never reserved (or allocated) a workspace
    ctx = nb.Context(0)
    q = synth.random_positive(300, 500, 33, seed=811, zeros=0.1)
    V, W, H = dev(q.V), dev(q.W), dev(q.H)
    o = torch.zeros(1, dtype=torch.float64, device=DEV)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        assert noalloc(ctx, V, W, H, 1.0, "joint", obj=o, stream=s) == 0
    We, He = dev(q.W), dev(q.H)
    oe = torch.zeros(1, dtype=torch.float64, device=DEV)
    nb.step(V, We, He, 1.0, "joint", objective_out=oe, ctx=nb.Context(0))
    torch.cuda.synchronize()
    for rep in range(3):
        W.copy_(dev(q.W))
        H.copy_(dev(q.H))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(W, We) and torch.equal(H, He), rep
        assert o.item() == oe.item(), rep
        # eager no-allocation work between replays, on another shape
        r = synth.random_positive(90, 120, 7, seed=812 + rep)
        assert noalloc(ctx, dev(r.V), dev(r.W), dev(r.H), 2.0, "alternating") == 0
        torch.cuda.synchronize()
    del g
    ctx.close()


def test_noalloc_rejects_oversized_step_and_reports_flags():
    ctx = nb.Context(0)
    # joint sub-iterations need the kept P, Q tiles: 2048 x 4096, K = 64 does
    # not fit in the scratch array -> rejected on the host, nothing launched
    F, N, K = 2048, 4096, 64
    V = torch.ones(F, N, device=DEV)
    W = torch.ones(F, K, device=DEV)
    H = torch.ones(K, N, device=DEV)
    assert noalloc(ctx, V, W, H, 1.0, "joint", inner_iters=2) == NMF_ERR_WORKSPACE
    with pytest.raises(nb.NmfError):
        nb.step_noalloc(V, W, H, 1.0, "joint", inner_iters=2, ctx=ctx)
    assert torch.all(W == 1) and torch.all(H == 1)
    # the same shape at L = 1 fits without the kept tiles and matches nmf_beta_step
    p = synth.random_positive(F, N, K, seed=813)
    V = dev(p.V)
    Wa, Ha, Wb, Hb = dev(p.W), dev(p.H), dev(p.W), dev(p.H)
    assert noalloc(ctx, V, Wa, Ha, 1.0, "joint") == 0
    nb.step(V, Wb, Hb, 1.0, "joint", ctx=ctx)
    torch.cuda.synchronize()
    Wr, Hr = O.jmm_iteration(p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64), 1.0)
    check_pair(Wa.cpu().numpy(), Ha.cpu().numpy(), Wr, Hr, tag="noalloc without kept P/Q")
    check_pair(Wb.cpu().numpy(), Hb.cpu().numpy(), Wr, Hr, tag="step with kept P/Q")
    # a zero H gives zero denominators: the flag lands in the caller's word
    q = synth.random_positive(64, 80, 6, seed=814)
    fl = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert noalloc(ctx, dev(q.V), dev(q.W), torch.zeros(6, 80, device=DEV), 1.0, "joint", flags=fl) == 0
    torch.cuda.synchronize()
    assert fl.item() & nb.FLAG_NONFINITE
    ctx.close()
