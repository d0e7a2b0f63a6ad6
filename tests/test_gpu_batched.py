"""GPU parity of the batched persistent step (many uneven problems, each with
its own beta and rank, one launch per outer iteration) against the FP64 oracle
and against the single-problem step.

Gates as for the single-problem path (tests/gates.py): W, H relative Frobenius
error <= 1e-5 and entry-wise <= 1e-4 (float32), or 3e-3 and 4 u (2 + |beta - 2|)
(bfloat16, u = 2^-9); objective <= 1e-6 (float32 Lambda).  Against the
single-problem step (same arithmetic, other split of the reductions) <= 2e-6;
those runs are also compared with the oracle.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth
import paper_2106_15214_amd as nb
from gates import check_pair, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = nb.Context(0)
        _CTX["c"].set_path("stream")
    return _CTX["c"]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# uneven shapes, ranks on both sides of 32, every beta class
SPECS = [(64, 100, 5, 1.0), (200, 150, 20, 0.0), (257, 300, 49, 0.5), (130, 70, 64, 2.0), (33, 1000, 8, 1.5),
         (1, 40, 3, 1.2), (40, 1, 3, 2.5), (129, 129, 1, -0.5), (96, 160, 32, 1.0), (300, 97, 33, 0.0),
         (500, 260, 17, 2.0), (77, 611, 60, 0.5)]


# problems with K < min(F, N): several steps stay away from an exact fit, after
# which the update ratio is the undefined 0/0 (flagged by every path)
WELL_POSED = [s for s in SPECS if s[2] < min(s[0], s[1])]


def make_set(specs, seed0=100):
    out = []
    for i, (F, N, K, beta) in enumerate(specs):
        p = synth.random_positive(F, N, K, seed=seed0 + i, zeros=0.1 if beta > 0 else 0.0)
        out.append((p.V, p.W, p.H, beta))
    return out


def to_dev(probs):
    return [(dev(V), dev(W), dev(H), b) for V, W, H, b in probs]


def oracle_step(V, W, H, beta, mode):
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    return f(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta)


# tiles 0: the context's table (every problem here one group per pass: in
# float32 no update phases); 1, 3: several groups (all four phases); 12: a mix
# of both and of problems that skip only the W-update phase (F = 500: two row
# groups, N = 260: one column group)
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("tiles", [0, 1, 3, 12])
def test_batched_step_matches_oracle(mode, tiles):
    probs = make_set(SPECS)
    d = to_dev(probs)
    print(f"[batched] mode={mode} tiles={tiles} problems={len(d)}", flush=True)
    b = nb.Batch(d, mode, tiles_per_item=tiles, ctx=ctx())
    obj = torch.full((len(d),), float("nan"), dtype=torch.float64, device=DEV)
    b.step(objectives=obj)
    torch.cuda.synchronize()
    assert b.flags(clear=True) == 0
    o = obj.cpu().numpy()
    for i, ((V, W, H, beta), (_, Wd, Hd, _)) in enumerate(zip(probs, d)):
        Wr, Hr = oracle_step(V, W, H, beta, mode)
        d0 = O.objective(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta)
        check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=f"problem {i} {V.shape} K={W.shape[1]} beta={beta}")
        assert abs(o[i] - d0) <= 1e-6 * abs(d0), (i, o[i], d0)
    b.close()


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_batched_several_steps_match_single_problem_steps(mode):
    probs = make_set(WELL_POSED, seed0=300)
    d = to_dev(probs)
    ref = to_dev(probs)
    b = nb.Batch(d, mode, ctx=ctx())
    obj = torch.zeros(len(d), dtype=torch.float64, device=DEV)
    o1 = torch.zeros(1, dtype=torch.float64, device=DEV)
    for t in range(6):
        b.step(objectives=obj)
        ob = obj.cpu().numpy()
        for i, (V, W, H, beta) in enumerate(ref):
            nb.step(V, W, H, beta, mode, objective_out=o1, ctx=ctx())
            assert abs(ob[i] - o1.item()) <= 2e-6 * abs(o1.item()) + 1e-10, (t, i)
    torch.cuda.synchronize()
    assert b.flags() == 0 and nb.get_flags(clear=True, ctx=ctx()) == 0
    for i, ((_, Wb, Hb, _), (_, Wr, Hr, _)) in enumerate(zip(d, ref)):
        assert rel(Wb.cpu().numpy(), Wr.cpu().numpy().astype(np.float64)) <= 1e-5, i
        assert rel(Hb.cpu().numpy(), Hr.cpu().numpy().astype(np.float64)) <= 1e-5, i
    b.close()
    # the same six steps by the oracle: per-step bars times the number of steps
    for i, ((V, W, H, beta), (_, Wb, Hb, _)) in enumerate(zip(probs, d)):
        Wr, Hr = W.astype(np.float64), H.astype(np.float64)
        for _ in range(6):
            Wr, Hr = oracle_step(V, Wr, Hr, beta, mode)
        check_pair(Wb.cpu().numpy(), Hb.cpu().numpy(), Wr, Hr, tag=f"6 steps problem {i}", fro=6e-5, el=6e-4)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("tiles", [0, 1, 12])
def test_batch_items_match_requirements(precision, mode, tiles):
    """The host's requirements count exactly the work items a batch lists."""
    probs = to_dev(make_set(SPECS, seed0=550))
    shapes = [(V.shape[0], V.shape[1], W.shape[1], beta) for V, W, H, beta in probs]
    c = ctx()
    b = nb.Batch(probs, mode, precision=precision, tiles_per_item=tiles, ctx=c)
    table = [tiles] * nb.BATCH_BUCKETS if tiles else nb.get_batch_tiles(c)
    assert b.info()["work_items"] == nb.batch_requirements(shapes, mode, table, precision)[0]
    b.close()


# tiles as in test_batched_step_matches_oracle: folded updates, all four
# phases, and a mix (joint problems at K <= 32 or beta = 1 form Lambda~ again
# from a row-major copy of W~, the others keep P, Q)
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("tiles", [0, 1, 12])
def test_batched_bf16_matches_oracle(mode, tiles):
    specs = [s for s in SPECS]
    probs = make_set(specs, seed0=500)
    d = to_dev(probs)
    print(f"[batched bf16] mode={mode} tiles={tiles} problems={len(d)}", flush=True)
    b = nb.Batch(d, mode, precision="bf16", tiles_per_item=tiles, ctx=ctx())
    b.step()
    torch.cuda.synchronize()
    assert b.flags(clear=True) == 0
    for i, ((V, W, H, beta), (_, Wd, Hd, _)) in enumerate(zip(probs, d)):
        Wr, Hr = oracle_step(V, W, H, beta, mode)
        check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, "bf16", beta, tag=f"bf16 problem {i}")
    b.close()


def test_batched_graph_capture_replays_match_eager():
    probs = make_set(WELL_POSED, seed0=700)
    eager = to_dev(probs)
    graph = to_dev(probs)
    be = nb.Batch(eager, "joint", ctx=ctx())
    bg = nb.Batch(graph, "joint", ctx=ctx())
    oe = torch.zeros(len(probs), dtype=torch.float64, device=DEV)
    og = torch.zeros(len(probs), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bg.step(objectives=og)
    torch.cuda.synchronize()
    # capture does not run the kernel: both batches are still at the start
    for rep in range(4):
        be.step(objectives=oe)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(oe, og), rep
        for (_, We, He, _), (_, Wg, Hg, _) in zip(eager, graph):
            assert torch.equal(We, Wg) and torch.equal(He, Hg), rep
    assert be.flags() == 0 and bg.flags() == 0
    be.close()
    bg.close()


def test_batched_workload_sample_matches_single_steps():
    # 48 problems of the batched workload's draw (F, N scaled by 1/4)
    specs = synth.batched_specs(48)
    probs = []
    for sp in specs:
        p = synth.make_batched_problem(sp, scale=0.25)
        probs.append((p.V, p.W, p.H, p.beta))
    d = to_dev(probs)
    ref = to_dev(probs)
    b = nb.Batch(d, "joint", ctx=ctx())
    print(f"[batched] workload sample: {b.info()}", flush=True)
    obj = torch.zeros(len(d), dtype=torch.float64, device=DEV)
    b.step(objectives=obj)
    o1 = torch.zeros(1, dtype=torch.float64, device=DEV)
    ob = obj.cpu().numpy()
    for i, (V, W, H, beta) in enumerate(ref):
        nb.step(V, W, H, beta, "joint", objective_out=o1, ctx=ctx())
        assert abs(ob[i] - o1.item()) <= 2e-6 * abs(o1.item()) + 1e-10, i
    torch.cuda.synchronize()
    for i, ((_, Wb, Hb, _), (_, Wr, Hr, _)) in enumerate(zip(d, ref)):
        assert rel(Wb.cpu().numpy(), Wr.cpu().numpy().astype(np.float64)) <= 2e-6, i
        assert rel(Hb.cpu().numpy(), Hr.cpu().numpy().astype(np.float64)) <= 2e-6, i
    assert b.flags() == 0
    b.close()
    for i, ((V, W, H, beta), (_, Wb, Hb, _)) in enumerate(zip(probs, d)):
        Wr, Hr = oracle_step(V, W, H, beta, "joint")
        check_pair(Wb.cpu().numpy(), Hb.cpu().numpy(), Wr, Hr, tag=f"workload sample {i}")
        d0 = O.objective(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta)
        assert abs(ob[i] - d0) <= 1e-6 * abs(d0), i


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_batched_heuristic_exponent_matches_oracle(mode):
    probs = make_set(WELL_POSED, seed0=1300)
    d = to_dev(probs)
    b = nb.Batch(d, mode, exponent="one", ctx=ctx())
    b.step()
    torch.cuda.synchronize()
    assert b.flags() == 0
    b.close()
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    for i, ((V, W, H, beta), (_, Wd, Hd, _)) in enumerate(zip(probs, d)):
        Wr, Hr = f(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta, exponent="one")
        check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=str(i))


def test_batched_many_initializations_of_one_problem():
    # the evaluation protocol of Sec. 4.1.4: one V from 25 initializations, as one
    # batch whose problems share V (read-only); every problem against the oracle
    p = synth.make_problem("spectro_is", beta=0.5, rows=(0, 120), cols=(0, 700))
    V = dev(p.V)
    inits = []
    for seed in range(25):
        rng = np.random.default_rng(seed)
        inits.append((rng.uniform(0.1, 1.0, p.W.shape).astype(np.float32),
                      rng.uniform(0.1, 1.0, p.H.shape).astype(np.float32)))
    d = [(V, dev(W), dev(H), 0.5) for W, H in inits]
    b = nb.Batch(d, "joint", ctx=ctx())
    obj = torch.zeros(len(d), dtype=torch.float64, device=DEV)
    b.step(objectives=obj)
    torch.cuda.synchronize()
    assert b.flags() == 0
    b.close()
    V64 = p.V.astype(np.float64)
    ob = obj.cpu().numpy()
    for i, ((W, H), (_, Wd, Hd, _)) in enumerate(zip(inits, d)):
        W64, H64 = W.astype(np.float64), H.astype(np.float64)
        Wr, Hr = O.jmm_iteration(V64, W64, H64, 0.5)
        check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=str(i))
        d0 = O.objective(V64, W64, H64, 0.5)
        assert abs(ob[i] - d0) <= 1e-6 * abs(d0), i


def test_batched_rejects_aliasing_and_large_k():
    a, b = to_dev(make_set([(64, 100, 5, 1.0), (64, 100, 5, 0.5)], seed0=900))
    # the second problem updates the first one's W
    with pytest.raises(nb.NmfError):
        nb.Batch([a, (b[0], a[1], b[2], b[3])], "joint", ctx=ctx())
    # a problem's W inside another problem's V
    with pytest.raises(nb.NmfError):
        nb.Batch([a, (b[0], a[0][:, :5], b[2], b[3])], "joint", ctx=ctx())
    # V shared between problems is allowed (read-only)
    c = (a[0], a[1].clone(), a[2].clone(), 2.0)
    nb.Batch([a, c], "joint", ctx=ctx()).close()
    p = synth.random_positive(40, 50, 65, seed=3)
    with pytest.raises(nb.NmfError):
        nb.Batch([(dev(p.V), dev(p.W), dev(p.H), 1.0)], "joint", ctx=ctx())


def test_long_trajectory_kappa_reading():
    """Problem 152 of the batched workload (569 x 369, K = 8, beta = 0.5, Poisson V
    with about 40 % zeros): at kappa = 0 the iterates drive entries of WH to zero
    at the zeros of V until an update ratio is undefined, on the GPU and in the
    float64 oracle alike, near the same iteration; at kappa = 1e-9 (Sec. 4.1.3)
    both run 200 iterations with a non-increasing objective, and the GPU's
    objective trace follows the oracle's."""
    spec = synth.batched_specs(512)[152]
    q = synth.make_batched_problem(spec)
    assert spec["beta"] == 0.5 and np.mean(q.V == 0) > 0.3
    V64 = q.V.astype(np.float64)
    T = 200

    def oracle_run(kappa):
        W, H = q.W.astype(np.float64), q.H.astype(np.float64)
        trace = [O.objective(V64, W, H, 0.5, kappa=kappa)]
        for t in range(T):
            try:
                W, H = O.jmm_iteration(V64, W, H, 0.5, kappa=kappa)
            except FloatingPointError:
                return trace, t
            trace.append(O.objective(V64, W, H, 0.5, kappa=kappa))
        return trace, None

    def gpu_run(kappa):
        V, W, H = dev(q.V), dev(q.W), dev(q.H)
        b = nb.Batch([(V, W, H, 0.5)], "joint", kappa=kappa, ctx=ctx())
        tr = torch.zeros((T + 1, 1), dtype=torch.float64, device=DEV)
        first_flag = None
        for t in range(T + 1):
            b.step(objectives=tr[t])
            if first_flag is None and t % 5 == 4 and b.flags(clear=True):
                first_flag = t
        b.close()
        torch.cuda.synchronize()
        return tr[:, 0].cpu().numpy(), first_flag

    print("[batched] long trajectory, kappa = 0", flush=True)
    _, o_fail = oracle_run(0.0)
    g_trace, g_flag = gpu_run(0.0)
    assert o_fail is not None and g_flag is not None, (o_fail, g_flag)
    # the same breakdown near the same iteration (flags are polled every 5 steps)
    assert abs(g_flag - o_fail) <= 25, (g_flag, o_fail)

    print("[batched] long trajectory, kappa = 1e-9", flush=True)
    o_trace, o_fail = oracle_run(1e-9)
    g_trace, g_flag = gpu_run(1e-9)
    assert o_fail is None and g_flag is None, (o_fail, g_flag)
    g = g_trace[:T + 1]  # objective of iterates 0..T (the step at t reports iterate t)
    assert np.all(np.isfinite(g))
    assert np.all(np.diff(g) <= 1e-6 * g[1:]), "objective increased"
    o = np.asarray(o_trace)
    rel_dev = np.abs(g - o) / o
    print(f"[batched] trajectory deviation from the oracle: max {rel_dev.max():.2e}", flush=True)
    assert rel_dev.max() <= 1e-4
