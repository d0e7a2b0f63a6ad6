"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Every case starts both sides from the same float32 state.  Gates on the new
factors (tests/gates.py): relative Frobenius error <= 1e-5 and entry-wise
max |X - X_ref| / (|X_ref| + 1e-6 max|X_ref|) <= 1e-4 (float32 products);
relative objective error <= 1e-6.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synth
import paper_2106_15214_amd as nb
from gates import check_factor, check_pair, rel

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL_FACTOR = 1e-5
TOL_OBJ = 1e-6
BETAS = [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, -0.5, 1.2]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


_CTX = {}


def ctx_for(path):
    """One library context per execution path ("auto", "stream", "fused")."""
    if path not in _CTX:
        c = nb.Context(0)
        c.set_path(path)
        _CTX[path] = c
    return _CTX[path]


def gpu_step(V, W, H, beta, mode, kappa=0.0, normalize=True, obj=True, path="auto"):
    Vd, Wd, Hd = dev(V), dev(W), dev(H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV) if obj else None
    ctx = ctx_for(path)
    nb.step(Vd, Wd, Hd, beta, mode, kappa=kappa, normalize=normalize, objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    return Wd.cpu().numpy(), Hd.cpu().numpy(), (o.item() if obj else None)


def ref_step(V, W, H, beta, mode, kappa=0.0, normalize=True):
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    return f(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta, kappa=kappa, norm=normalize)


def ref_obj(V, W, H, beta, kappa=0.0):
    return O.objective(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta, kappa)


def check_step(V, W, H, beta, mode, kappa=0.0, normalize=True, tag="", path="auto"):
    print(f"[parity] {tag} F={V.shape[0]} N={V.shape[1]} K={W.shape[1]} beta={beta} mode={mode} "
          f"kappa={kappa} norm={normalize} path={path}", flush=True)
    Wg, Hg, dg = gpu_step(V, W, H, beta, mode, kappa, normalize, path=path)
    Wr, Hr = ref_step(V, W, H, beta, mode, kappa, normalize)
    d0 = ref_obj(V, W, H, beta, kappa)
    check_pair(Wg, Hg, Wr, Hr, tag=tag)
    eD = abs(dg - d0) / abs(d0)
    assert eD <= TOL_OBJ, f"objective rel err {eD:.3e} ({dg} vs {d0})"
    return Wg, Hg


SHAPES = [(64, 100, 5), (200, 150, 20), (257, 300, 49), (130, 70, 64), (33, 1000, 8), (1, 40, 3), (40, 1, 3),
          (300, 97, 100), (129, 129, 1), (96, 160, 32)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_step_parity_shapes(shape, beta, mode, path):
    F, N, K = shape
    if path == "fused" and K > 64:
        pytest.skip("the single-launch path covers K <= 64")
    p = synth.random_positive(F, N, K, seed=F * 7 + N + K, zeros=0.1 if beta > 0 else 0.0)
    check_step(p.V, p.W, p.H, beta, mode, tag="shape", path=path)


@pytest.mark.parametrize("name,beta,crop", [
    ("tiny_kl", 1.0, None),
    ("faces_euc", 2.0, None),
    ("spectro_is", 0.0, None),
    ("spectro_is", 0.5, None),
    ("counts_kl", 1.0, ((0, 200), (0, 150))),
    ("counts_kl", 1.0, ((1000, 1700), (3000, 4100))),
])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_workload_parity(name, beta, crop, mode, path):
    p = synth.make_problem(name, beta=beta, rows=crop[0] if crop else None, cols=crop[1] if crop else None)
    check_step(p.V, p.W, p.H, beta, mode, tag=name, path=path)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_trajectory_per_step_parity_tiny_kl(mode):
    # 100 iterations of the tiny KL workload; at selected t the GPU state is
    # stepped once by both sides; the objective trace is monotone.
    p = synth.make_problem("tiny_kl")
    V, W, H = dev(p.V), dev(p.W), dev(p.H)
    trace = []
    for t in range(100):
        if t in (0, 1, 10, 50, 99):
            check_step(p.V, W.cpu().numpy(), H.cpu().numpy(), 1.0, mode, tag=f"t={t}")
        o = torch.zeros(1, dtype=torch.float64, device=DEV)
        nb.step(V, W, H, 1.0, mode, objective_out=o)
        trace.append(o.item())
    trace = np.array(trace)
    eps = 2e-7  # objective evaluation error of the float32 product
    assert np.all(trace[1:] <= trace[:-1] * (1 + 2 * eps)), np.max(np.diff(trace) / trace[:-1])


@pytest.mark.parametrize("L", [2, 3])
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 2.0, 2.5])
@pytest.mark.parametrize("normalize", [True, False])
def test_alternating_sub_iterations_parity(L, beta, normalize):
    # Algorithm 1 with L_W = L_H = L: L W updates against the latest W, then L H updates
    p = synth.random_positive(257, 300, 20, seed=43, zeros=0.1 if beta > 0 else 0.0)
    print(f"[parity] alternating L={L} beta={beta} normalize={normalize}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, beta, "alternating", inner_iters=L, normalize=normalize, objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    Wr, Hr = O.bmm_iteration(V64, W64, H64, beta, L_W=L, L_H=L, norm=normalize)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr)
    d0 = ref_obj(p.V, p.W, p.H, beta)
    assert abs(o.item() - d0) <= TOL_OBJ * abs(d0)


@pytest.mark.parametrize("L", [2, 3])
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5, 2.0, 2.5])
@pytest.mark.parametrize("normalize", [True, False])
def test_joint_sub_iterations_parity(L, beta, normalize):
    # Algorithm 2 with L sub-iterations: later W steps contract the kept P, Q
    # with chi(H_l, H~); every step multiplies the tilde iterate
    p = synth.random_positive(257, 300, 20, seed=45, zeros=0.1 if beta > 0 else 0.0)
    print(f"[parity] joint L={L} beta={beta} normalize={normalize}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, beta, "joint", inner_iters=L, normalize=normalize, objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    Wr, Hr = O.jmm_iteration(V64, W64, H64, beta, L=L, norm=normalize)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr)
    d0 = ref_obj(p.V, p.W, p.H, beta)
    assert abs(o.item() - d0) <= TOL_OBJ * abs(d0)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_sub_iterations_large_rank(mode):
    # K = 100 (four 32-column blocks), ragged shape
    p = synth.random_positive(300, 197, 100, seed=46)
    print(f"[parity] sub-iterations K=100 mode={mode}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, 0.5, mode, inner_iters=3, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    if mode == "joint":
        Wr, Hr = O.jmm_iteration(V64, W64, H64, 0.5, L=3)
    else:
        Wr, Hr = O.bmm_iteration(V64, W64, H64, 0.5, L_W=3, L_H=3)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr)


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_alternating_sub_iterations_low_precision(precision, beta):
    # low-precision products: the per-step bar of the low-precision tests (3e-3)
    p = synth.random_positive(257, 300, 20, seed=47, zeros=0.1)
    print(f"[parity] alternating L=2 {precision} beta={beta}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, beta, "alternating", precision=precision, inner_iters=2, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    Wr, Hr = O.bmm_iteration(V64, W64, H64, beta, L_W=2, L_H=2)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, precision, beta)


def test_sub_iterations_rejected_where_unsupported():
    p = synth.random_positive(64, 80, 6, seed=44)
    with pytest.raises(nb.NmfError):
        nb.step(dev(p.V), dev(p.W), dev(p.H), 1.0, "joint", precision="bf16", inner_iters=2, ctx=ctx_for("auto"))
    for mode in ("joint", "alternating"):
        with pytest.raises(nb.NmfError):
            nb.step(dev(p.V), dev(p.W), dev(p.H), 1.0, mode, inner_iters=2, ctx=ctx_for("fused"))


@pytest.mark.parametrize("beta", [-0.5, 0.0, 0.5, 1.0, 2.5])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_heuristic_exponent_parity(beta, mode, path):
    # gamma = 1 for every beta (Sec. 3.3.3): the same passes with another exponent
    p = synth.random_positive(257, 300, 20, seed=41, zeros=0.1 if beta > 0 else 0.0)
    print(f"[parity] heuristic exponent beta={beta} mode={mode} path={path}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    ctx = ctx_for(path)
    nb.step(Vd, Wd, Hd, beta, mode, exponent="one", objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    Wr, Hr = f(V64, W64, H64, beta, exponent="one")
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr)
    d0 = ref_obj(p.V, p.W, p.H, beta)
    assert abs(o.item() - d0) <= TOL_OBJ * abs(d0)


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0, 0.5])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_w_step_bitwise_equal_between_modes(beta, path):
    p = synth.random_positive(150, 190, 24, seed=3)
    Wj, _, _ = gpu_step(p.V, p.W, p.H, beta, "joint", path=path)
    Wa, _, _ = gpu_step(p.V, p.W, p.H, beta, "alternating", path=path)
    assert np.array_equal(Wj, Wa)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_run_to_run_bitwise_determinism(mode, path):
    p = synth.random_positive(300, 500, 50, seed=4)
    a = gpu_step(p.V, p.W, p.H, 1.5, mode, path=path)
    b = gpu_step(p.V, p.W, p.H, 1.5, mode, path=path)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


@pytest.mark.parametrize("beta", [0.0, 1.0, 2.0])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_paths_agree(beta, mode):
    # the single launch and the four launches compute the same update (to rounding)
    p = synth.random_positive(230, 410, 33, seed=21)
    a = gpu_step(p.V, p.W, p.H, beta, mode, path="stream")
    b = gpu_step(p.V, p.W, p.H, beta, mode, path="fused")
    assert rel(b[0], a[0].astype(np.float64)) <= 2e-6 and rel(b[1], a[1].astype(np.float64)) <= 2e-6
    assert abs(a[2] - b[2]) <= 1e-12 * abs(a[2])


def test_fused_path_refuses_large_k():
    p = synth.random_positive(40, 50, 100, seed=22)
    with pytest.raises(nb.NmfError):
        gpu_step(p.V, p.W, p.H, 1.0, "joint", path="fused")


@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("beta", [0.0, 1.0])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_kappa_smoothing_with_zeros(mode, beta, path):
    p = synth.random_positive(120, 140, 10, seed=5, zeros=0.3)
    check_step(p.V, p.W, p.H, beta, mode, kappa=0.05, tag="kappa", path=path)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("path", ["stream", "fused"])
def test_without_normalization(mode, path):
    p = synth.random_positive(100, 140, 12, seed=6)
    check_step(p.V, p.W, p.H, 0.5, mode, normalize=False, tag="nonorm", path=path)


def test_padded_leading_dimensions_and_unaligned_v():
    p = synth.random_positive(90, 130, 17, seed=8)
    big = np.zeros((90, 133), np.float32)
    big[:, 1:131] = p.V  # V starts one float in: rows not 16-byte aligned
    Vd = dev(big)[:, 1:131]
    Wb = np.zeros((90, 21), np.float32)
    Wb[:, :17] = p.W
    Hb = np.zeros((17, 140), np.float32)
    Hb[:, :130] = p.H
    Wbig, Hbig = dev(Wb), dev(Hb)
    Wd = Wbig[:, :17]
    Hd = Hbig[:, :130]
    o = torch.zeros(1, dtype=torch.float64, device=DEV)
    nb.step(Vd, Wd, Hd, 1.0, "joint", objective_out=o)
    torch.cuda.synchronize()
    Wr, Hr = ref_step(p.V, p.W, p.H, 1.0, "joint")
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr)
    # padding columns untouched
    assert torch.all(Wbig[:, 17:] == 0) and torch.all(Hbig[:, 130:] == 0)
    assert abs(o.item() - ref_obj(p.V, p.W, p.H, 1.0)) <= TOL_OBJ * ref_obj(p.V, p.W, p.H, 1.0)


@pytest.mark.parametrize("beta", BETAS + [3.0])
@pytest.mark.parametrize("kappa", [0.0, 0.1])
def test_objective_call(beta, kappa):
    p = synth.random_positive(170, 230, 19, seed=9, zeros=0.1 if (beta > 0 or kappa > 0) else 0.0)
    out = nb.objective(dev(p.V), dev(p.W), dev(p.H), beta, kappa=kappa)
    d0 = ref_obj(p.V, p.W, p.H, beta, kappa)
    assert abs(out.item() - d0) <= TOL_OBJ * abs(d0)


def _grad_tol_scale(V, W, H, beta):
    L = W.astype(np.float64) @ H.astype(np.float64)
    E = np.abs(L ** (beta - 2) * (L - V))
    return np.linalg.norm(E @ np.abs(H.T)), np.linalg.norm(np.abs(W.T) @ E)


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5, 2.0, 2.5])
def test_gradient_matches_oracle(beta):
    p = synth.random_positive(150, 260, 30, seed=10)
    dW, dH = nb.grad(dev(p.V), dev(p.W), dev(p.H), beta, scale=1.0)
    gW, gH = O.gradient(p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64), beta)
    sW, sH = _grad_tol_scale(p.V, p.W, p.H, beta)
    assert np.linalg.norm(dW.cpu().numpy() - gW) <= 1e-5 * sW
    assert np.linalg.norm(dH.cpu().numpy() - gH) <= 1e-5 * sH


def test_gradient_count_crop_finite_differences_and_autograd():
    # count-data crop V[:200, :150], K = 50: GPU autograd backward vs the oracle
    # gradient and vs central finite differences of the oracle objective
    p = synth.make_problem("counts_kl", rows=(0, 200), cols=(0, 150))
    V, W, H = dev(p.V), dev(p.W).requires_grad_(True), dev(p.H).requires_grad_(True)
    D = nb.beta_divergence(V, W, H, 1.0)
    (3.0 * D).backward()
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    gW, gH = O.gradient(V64, W64, H64, 1.0)
    sW, sH = _grad_tol_scale(p.V, p.W, p.H, 1.0)
    assert np.linalg.norm(W.grad.cpu().numpy() - 3.0 * gW) <= 3e-5 * sW
    assert np.linalg.norm(H.grad.cpu().numpy() - 3.0 * gH) <= 3e-5 * sH
    rng = np.random.default_rng(0)
    for _ in range(10):
        f, k = rng.integers(0, 200), rng.integers(0, 50)
        h = 1e-6 * max(1.0, W64[f, k])
        Wp, Wm = W64.copy(), W64.copy()
        Wp[f, k] += h
        Wm[f, k] -= h
        fd = (O.objective(V64, Wp, H64, 1.0) - O.objective(V64, Wm, H64, 1.0)) / (2 * h)
        assert abs(W.grad[f, k].item() / 3.0 - fd) <= 1e-4 * max(1.0, abs(fd))
    assert abs(D.item() - O.objective(V64, W64, H64, 1.0)) <= TOL_OBJ * O.objective(V64, W64, H64, 1.0)


def test_flags_nonfinite_and_domain():
    nb.get_flags(clear=True)
    p = synth.random_positive(64, 80, 6, seed=11)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    nb.validate(Vd, Wd, Hd, 1.0)
    assert nb.get_flags(clear=True) == 0
    Vbad = p.V.copy()
    Vbad[3, 4] = -1.0
    nb.validate(dev(Vbad), Wd, Hd, 1.0)
    assert nb.get_flags(clear=True) & nb.FLAG_DOMAIN
    Vz = p.V.copy()
    Vz[0, 0] = 0.0
    nb.validate(dev(Vz), Wd, Hd, 0.0)
    assert nb.get_flags(clear=True) & nb.FLAG_DOMAIN
    nb.validate(dev(Vz), Wd, Hd, 0.0, kappa=0.1)
    assert nb.get_flags(clear=True) == 0
    for path in ("stream", "fused"):
        ctx = ctx_for(path)
        Hz = torch.zeros_like(Hd)
        nb.step(Vd, Wd.clone(), Hz, 1.0, "joint", ctx=ctx)
        assert nb.get_flags(clear=True, ctx=ctx) & nb.FLAG_NONFINITE
        assert nb.get_flags(ctx=ctx) == 0


def test_workspace_regrowth_between_sizes():
    for (F, N, K) in [(50, 60, 4), (700, 900, 70), (40, 30, 2), (1200, 300, 33)]:
        p = synth.random_positive(F, N, K, seed=F + N)
        check_step(p.V, p.W, p.H, 1.0, "joint", tag="regrow")


@pytest.mark.parametrize("mode,L", [("joint", 2), ("alternating", 3)])
def test_sub_iterations_under_graph_capture(mode, L):
    # after nmf_reserve a step with L sub-iterations allocates nothing and can be
    # captured; every replay (with eager work between them) matches the oracle
    ctx = nb.Context(0)
    ctx.reserve(400, 500, 40)
    q = synth.random_positive(150, 333, 17, seed=14)
    print(f"[parity] graph capture mode={mode} L={L}", flush=True)
    Vq, Wq, Hq = dev(q.V), dev(q.W), dev(q.H)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        nb.step(Vq, Wq, Hq, 0.5, mode, inner_iters=L, ctx=ctx, stream=s)
    V64, W64, H64 = (a.astype(np.float64) for a in (q.V, q.W, q.H))
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    Wr, Hr = f(V64, W64, H64, 0.5, L=L) if mode == "joint" else f(V64, W64, H64, 0.5, L_W=L, L_H=L)
    for rep in range(3):
        Wq.copy_(dev(q.W))
        Hq.copy_(dev(q.H))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check_pair(Wq.cpu().numpy(), Hq.cpu().numpy(), Wr, Hr, tag=f"replay {rep}")
        # eager work between the replays
        We, He = dev(q.W), dev(q.H)
        nb.step(Vq, We, He, 0.5, mode, inner_iters=L, ctx=ctx)
        torch.cuda.synchronize()
        check_factor(We.cpu().numpy(), Wr, what=f"W eager {rep}")
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    ctx.close()


def test_reserve_then_steps_do_not_allocate():
    ctx = nb.Context(0)
    ctx.reserve(400, 500, 40)
    p = synth.random_positive(400, 500, 40, seed=12)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    nb.step(Vd, Wd, Hd, 2.0, "joint", ctx=ctx)
    torch.cuda.synchronize()
    Wr, Hr = ref_step(p.V, p.W, p.H, 2.0, "joint")
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr)
    # a smaller problem inside the reservation must also work while capturing
    q = synth.random_positive(100, 333, 17, seed=13)
    Vq, Wq, Hq = dev(q.V), dev(q.W), dev(q.H)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        nb.step(Vq, Wq, Hq, 1.0, "joint", ctx=ctx, stream=s)
    Wq.copy_(dev(q.W))
    Hq.copy_(dev(q.H))
    g.replay()
    torch.cuda.synchronize()
    Wr, Hr = ref_step(q.V, q.W, q.H, 1.0, "joint")
    check_pair(Wq.cpu().numpy(), Hq.cpu().numpy(), Wr, Hr)
    ctx.close()


@pytest.mark.parametrize("K", [49, 64])
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 2.0])
def test_joint_sub_iterations_two_column_blocks(K, beta):
    # K in (32, 64]: the kept-P/Q W pass of later sub-iterations with two
    # 32-column blocks of the contraction (ragged at K = 49)
    p = synth.random_positive(190, 261, K, seed=48 + K, zeros=0.1 if beta > 0 else 0.0)
    print(f"[parity] joint L=2 K={K} beta={beta}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, beta, "joint", inner_iters=2, objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    Wr, Hr = O.jmm_iteration(V64, W64, H64, beta, L=2)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=f"joint L=2 K={K}")
    d0 = ref_obj(p.V, p.W, p.H, beta)
    assert abs(o.item() - d0) <= TOL_OBJ * abs(d0)


@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_joint_sub_iterations_with_kappa(beta):
    p = synth.random_positive(150, 170, 40, seed=61, zeros=0.3)
    print(f"[parity] joint L=3 kappa=0.05 beta={beta}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, beta, "joint", inner_iters=3, kappa=0.05, objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    V64, W64, H64 = (a.astype(np.float64) for a in (p.V, p.W, p.H))
    Wr, Hr = O.jmm_iteration(V64, W64, H64, beta, L=3, kappa=0.05)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag="joint L=3 kappa")
    d0 = ref_obj(p.V, p.W, p.H, beta, 0.05)
    assert abs(o.item() - d0) <= TOL_OBJ * abs(d0)


def test_binding_rejects_overlapping_rows_and_bad_objective_buffers():
    p = synth.random_positive(20, 30, 4, seed=62)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    Vx = Vd[:1].expand(20, 30)  # stride 0 rows: no valid leading dimension
    with pytest.raises(ValueError):
        nb.step(Vx, Wd, Hd, 1.0, "joint")
    with pytest.raises(ValueError):
        nb.step(Vd, Wd, Hd, 1.0, "joint", objective_out=torch.zeros(1, dtype=torch.float32, device=DEV))
    with pytest.raises(ValueError):
        nb.step(Vd, Wd, Hd, 1.0, "joint", objective_out=torch.zeros(0, dtype=torch.float64, device=DEV))
    with pytest.raises(ValueError):
        nb.grad(Vd, Wd, Hd, 1.0, objective_out=torch.zeros(1, dtype=torch.float64))  # host tensor
    # nothing ran: the factors are untouched
    assert torch.equal(Wd, dev(p.W)) and torch.equal(Hd, dev(p.H))


def test_workspace_does_not_move_after_capture():
    # a captured graph points into the workspace: a later call needing more
    # workspace is refused instead of freeing it (the graph is not replayed here)
    ctx = nb.Context(0)
    ctx.reserve(100, 120, 8)
    q = synth.random_positive(100, 120, 8, seed=63)
    Vq, Wq, Hq = dev(q.V), dev(q.W), dev(q.H)
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        nb.step(Vq, Wq, Hq, 1.0, "joint", ctx=ctx, stream=s)
    big = synth.random_positive(600, 700, 40, seed=64)
    with pytest.raises(nb.NmfError) as ei:
        nb.step(dev(big.V), dev(big.W), dev(big.H), 1.0, "joint", ctx=ctx)
    assert ei.value.status == 5  # NMF_ERR_WORKSPACE
    with pytest.raises(nb.NmfError):
        ctx.reserve(600, 700, 40)
    # calls within the reservation still run eagerly
    Wr, Hr = ref_step(q.V, q.W, q.H, 1.0, "joint")
    We, He = dev(q.W), dev(q.H)
    nb.step(Vq, We, He, 1.0, "joint", ctx=ctx)
    torch.cuda.synchronize()
    check_pair(We.cpu().numpy(), He.cpu().numpy(), Wr, Hr, tag="after capture")
    del g
    ctx.close()


def test_autograd_backward_uses_device_scale():
    # the upstream gradient reaches the library as a device scalar; a graph of
    # the backward's library calls is therefore possible (no host read)
    p = synth.random_positive(60, 70, 6, seed=65)
    V, W, H = dev(p.V), dev(p.W).requires_grad_(True), dev(p.H).requires_grad_(True)
    D = nb.beta_divergence(V, W, H, 0.5)
    (D * torch.tensor(2.5, dtype=torch.float64, device=DEV)).backward()
    gW, gH = O.gradient(p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64), 0.5)
    sW, sH = _grad_tol_scale(p.V, p.W, p.H, 0.5)
    assert np.linalg.norm(W.grad.cpu().numpy() - 2.5 * gW) <= 3e-5 * sW
    assert np.linalg.norm(H.grad.cpu().numpy() - 2.5 * gH) <= 3e-5 * sH


GRAM_SHAPES = [(64, 100, 5), (257, 300, 49), (130, 70, 64), (33, 1000, 8), (1, 40, 3), (40, 1, 3), (129, 129, 1),
               (361, 2429, 49)]


@pytest.mark.parametrize("shape", GRAM_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("obj", [True, False])
def test_gram_form_beta2_parity(shape, mode, obj):
    # beta = 2 with the Gram-form denominators of Table 2: the same iteration as
    # the oracle's (whose beta = 2 step is pinned to the textbook Gram-form rules)
    F, N, K = shape
    p = synth.random_positive(F, N, K, seed=F + 2 * N + K, zeros=0.1)
    print(f"[parity] gram F={F} N={N} K={K} mode={mode} obj={obj}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV) if obj else None
    ctx = ctx_for("auto")
    nb.step(Vd, Wd, Hd, 2.0, mode, gram=True, objective_out=o, ctx=ctx)
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx) == 0
    Wr, Hr = ref_step(p.V, p.W, p.H, 2.0, mode)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=f"gram {mode}")
    if obj:
        d0 = ref_obj(p.V, p.W, p.H, 2.0)
        assert abs(o.item() - d0) <= TOL_OBJ * abs(d0)


def test_gram_form_trajectory_matches_contraction_form():
    p = synth.make_problem("faces_euc")
    V = dev(p.V)
    Wa, Ha, Wb, Hb = dev(p.W), dev(p.H), dev(p.W), dev(p.H)
    oa = torch.zeros(1, dtype=torch.float64, device=DEV)
    ob = torch.zeros(1, dtype=torch.float64, device=DEV)
    ta, tb = [], []
    for _ in range(50):
        nb.step(V, Wa, Ha, 2.0, "joint", gram=True, objective_out=oa)
        nb.step(V, Wb, Hb, 2.0, "joint", objective_out=ob)
        ta.append(oa.item())
        tb.append(ob.item())
    assert nb.get_flags(clear=True) == 0
    assert np.all(np.diff(ta) <= 2e-7 * np.abs(ta[1:]))
    assert np.allclose(ta, tb, rtol=1e-5)
    check_pair(Wa.cpu().numpy(), Ha.cpu().numpy(), Wb.cpu().numpy().astype(np.float64),
               Hb.cpu().numpy().astype(np.float64), tag="gram vs contraction after 50 steps", fro=1e-4, el=1e-3)


def test_gram_form_rejected_where_unsupported():
    p = synth.random_positive(40, 50, 6, seed=66)
    V, W, H = dev(p.V), dev(p.W), dev(p.H)
    for kw in (dict(beta=1.0), dict(beta=2.0, kappa=0.1), dict(beta=2.0, precision="bf16"),
               dict(beta=2.0, inner_iters=2)):
        beta = kw.pop("beta")
        with pytest.raises(nb.NmfError):
            nb.step(V, W, H, beta, "joint", gram=True, **kw)
    q = synth.random_positive(40, 50, 65, seed=67)
    with pytest.raises(nb.NmfError):
        nb.step(dev(q.V), dev(q.W), dev(q.H), 2.0, "joint", gram=True)
    assert torch.equal(W, dev(p.W))
