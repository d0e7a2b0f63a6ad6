"""The device-side outer loop (nmf_beta_run: objective trace and the stopping
rule of Sec. 4.1.2 on the device) and the KKT residuals of Sec. 4.1.5
(nmf_beta_kkt), against the FP64 oracle.

* KKT residuals: |res_gpu - res_oracle| <= 1e-5 * (sum |E| |H|^T) / (F K) (and the
  same for H with |W|^T |E|): the condition-scaled bar of the gradient, whose
  entries the residuals take the minimum with; plus 1e-6 relative.
* Runs: the trace equals the objectives of eager steps bitwise (same kernels),
  matches the oracle's trajectory within 1e-5 relative, and the stop iteration
  is the oracle's stop_iteration() of the GPU's own trace (the rule is
  applied exactly); against the oracle's trajectory it is equal where the
  oracle's relative decrease is well separated from eps, else within one.
  W, H after the run equal the iterate at the stop.  A run captured in a HIP
  graph and replayed (with eager work between replays) repeats the eager run.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth
import paper_2106_15214_amd as nb

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = nb.Context(0)
    return _CTX["c"]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5, 2.0, 2.5])
@pytest.mark.parametrize("shape", [(120, 170, 9), (257, 300, 49), (40, 1, 3), (300, 97, 100)],
                         ids=lambda s: "x".join(map(str, s)))
def test_kkt_residuals_match_oracle(beta, shape):
    F, N, K = shape
    p = synth.random_positive(F, N, K, seed=F + N + K, zeros=0.1 if beta > 0 else 0.0)
    print(f"[kkt] F={F} N={N} K={K} beta={beta}", flush=True)
    r = nb.kkt(dev(p.V), dev(p.W), dev(p.H), beta, ctx=ctx()).cpu().numpy()
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    rW, rH = O.kkt_residuals(V64, W64, H64, beta)
    L = W64 @ H64
    E = np.abs(L ** (beta - 2.0) * (L - V64))
    sW = np.sum(E @ np.abs(H64.T)) / (F * K)
    sH = np.sum(np.abs(W64.T) @ E) / (K * N)
    assert abs(r[0] - rW) <= 1e-5 * sW + 1e-6 * abs(rW), (r[0], rW, sW)
    assert abs(r[1] - rH) <= 1e-5 * sH + 1e-6 * abs(rH), (r[1], rH, sH)


def test_kkt_residuals_fall_along_a_run():
    # the residuals of the iterates of a run decrease overall (first-order
    # optimality approached), GPU and oracle alike
    p = synth.make_problem("tiny_kl")
    V, W, H = dev(p.V), dev(p.W), dev(p.H)
    r0 = nb.kkt(V, W, H, 1.0, ctx=ctx()).cpu().numpy()
    for _ in range(100):
        nb.step(V, W, H, 1.0, "joint", ctx=ctx())
    r1 = nb.kkt(V, W, H, 1.0, ctx=ctx()).cpu().numpy()
    assert r1[0] < r0[0] and r1[1] < r0[1]
    rr = O.kkt_residuals(p.V.astype(np.float64), W.cpu().numpy().astype(np.float64),
                         H.cpu().numpy().astype(np.float64), 1.0)
    assert np.allclose(r1, rr, rtol=1e-3, atol=1e-7)


def oracle_trace(V, W, H, beta, mode, T):
    step = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    V64, W64, H64 = (a.astype(np.float64) for a in (V, W, H))
    tr = [O.objective(V64, W64, H64, beta)]
    for _ in range(T):
        W64, H64 = step(V64, W64, H64, beta)
        tr.append(O.objective(V64, W64, H64, beta))
    return np.array(tr)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("beta,eps", [(1.0, 1e-3), (0.5, 1e-3), (2.0, 1e-4), (0.0, 1e-3)])
def test_run_stop_rule_matches_oracle_and_eager_steps(mode, beta, eps):
    T = 150
    p = synth.random_positive(90, 130, 6, seed=77, zeros=0.1 if beta > 0 else 0.0)
    print(f"[run] mode={mode} beta={beta} eps={eps}", flush=True)
    V = dev(p.V)
    W, H = dev(p.W), dev(p.H)
    trace, stop = nb.run(V, W, H, beta, mode, max_iters=T, eps=eps, ctx=ctx())
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    tr = trace.cpu().numpy()
    t_stop = int(stop.item())
    # the rule applied exactly to the device trace
    assert t_stop == (O.stop_iteration(tr[: T + 1][np.isfinite(tr[: T + 1])], eps) or -1)
    assert t_stop > 0, "the rule should fire within the run for these tolerances"
    assert np.all(np.isnan(tr[t_stop + 1:]))
    # eager steps with the objective of every iterate: bitwise the same trace
    We, He = dev(p.W), dev(p.H)
    o = torch.zeros(1, dtype=torch.float64, device=DEV)
    eager = []
    for t in range(t_stop + 1):
        if t < t_stop:
            nb.step(V, We, He, beta, mode, objective_out=o, ctx=ctx())
        else:
            nb.objective(V, We, He, beta, out=o, ctx=ctx())
        eager.append(o.item())
    assert np.array_equal(np.array(eager), tr[: t_stop + 1])
    assert torch.equal(We, W) and torch.equal(He, H)
    # the oracle's trajectory: objective within 1e-5, stop where well separated
    ref = oracle_trace(p.V, p.W, p.H, beta, mode, min(T, t_stop + 2))
    assert np.allclose(tr[: t_stop + 1], ref[: t_stop + 1], rtol=1e-5, atol=0)
    s_ref = O.stop_iteration(ref, eps)
    assert s_ref is not None
    rd = (ref[:-1] - ref[1:]) / ref[1:]
    if rd[s_ref - 1] < 0.5 * eps and rd[s_ref - 2] > 2 * eps:
        assert t_stop == s_ref
    else:
        assert abs(t_stop - s_ref) <= 1


def test_run_without_stop_and_zero_iterations():
    p = synth.random_positive(60, 80, 5, seed=78)
    V, W, H = dev(p.V), dev(p.W), dev(p.H)
    trace, stop = nb.run(V, W, H, 1.0, "joint", max_iters=20, eps=-1e300, ctx=ctx())
    tr = trace.cpu().numpy()
    assert int(stop.item()) == -1 and np.all(np.isfinite(tr))
    ref = oracle_trace(p.V, p.W, p.H, 1.0, "joint", 20)
    assert np.allclose(tr, ref, rtol=1e-5, atol=0)
    W0 = W.clone()
    trace, stop = nb.run(V, W, H, 1.0, "joint", max_iters=0, ctx=ctx())
    assert int(stop.item()) == -1 and torch.equal(W, W0)
    assert abs(trace.item() - tr[-1]) <= 1e-12 * abs(tr[-1])


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_run_captured_in_a_graph(mode):
    c = nb.Context(0)
    p = synth.random_positive(150, 210, 12, seed=79, zeros=0.1)
    c.reserve(150, 210, 12)
    V, W, H = dev(p.V), dev(p.W), dev(p.H)
    T = 80
    trace = torch.full((T + 1,), float("nan"), dtype=torch.float64, device=DEV)
    stop = torch.zeros(1, dtype=torch.int32, device=DEV)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        nb.run(V, W, H, 0.5, mode, max_iters=T, eps=1e-3, trace=trace, stop=stop, ctx=c, stream=s)
    We, He = dev(p.W), dev(p.H)
    te, se = nb.run(V, We, He, 0.5, mode, max_iters=T, eps=1e-3, ctx=c)
    torch.cuda.synchronize()
    for rep in range(3):
        W.copy_(dev(p.W))
        H.copy_(dev(p.H))
        trace.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(stop.item()) == int(se.item()) > 0, rep
        assert np.array_equal(np.nan_to_num(trace.cpu().numpy(), nan=-1.0), np.nan_to_num(te.cpu().numpy(), nan=-1.0))
        assert torch.equal(W, We) and torch.equal(H, He), rep
        nb.step(V, dev(p.W), dev(p.H), 1.0, mode, ctx=c)  # eager work between replays
        torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=c) == 0
    del g
    c.close()
