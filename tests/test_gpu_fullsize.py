"""GPU parity at the benchmark workloads' full sizes, against the FP64 oracle.

* The 20000 x 10000 (K = 50, beta = 1) count workload: one outer iteration on
  the whole matrix, every entry of W and H compared entry-wise (and in
  Frobenius norm), and the objective and gradient calls, in the launch
  configuration the benchmark times (V is 800 MB, larger than the cache).
* A joint step just above 2^28 entries of V (16449 x 16353, ragged edges,
  beta = 0.5): beyond that size the joint step does not keep the P and Q tiles,
  and its H pass forms Lambda~ and its powers again from V, W~, H~.  Float32
  and bfloat16 products, every entry of W and H compared.
* The 512-problem batched workload at full size, in one persistent launch:
  every problem compared with the oracle, problem by problem.

Gates as in the other parity tests (tests/gates.py): float32 products W, H
<= 1e-5 relative (Frobenius) and <= 1e-4 entry-wise, objective <= 1e-6;
bfloat16 products W, H <= 3e-3 and 4 u (2 + |beta - 2|) entry-wise
(u = 2^-9), the objective within max(1e-6 D, 2^-14 S) (S: first-order change
of D under a 2^-14 relative change of every Lambda entry).
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth
import paper_2106_15214_amd as nb
from gates import check_pair

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = nb.Context(0)
    return _CTX["c"]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def counts():
    p = synth.make_problem("counts_kl")
    return p


def lowp_obj_bound(V64, W64, H64, beta):
    L = W64 @ H64
    return 2.0 ** -14 * float(np.sum(np.abs(L ** (beta - 1.0) * (L - V64))))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode,precision", [("joint", "fp32"), ("alternating", "fp32"), ("joint", "bf16")])
def test_count_workload_full_size(counts, mode, precision):
    p = counts
    F, N = p.V.shape
    K = p.W.shape[1]
    print(f"[fullsize] counts_kl F={F} N={N} K={K} beta={p.beta} mode={mode} precision={precision}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    nb.step(Vd, Wd, Hd, p.beta, mode, precision=precision, objective_out=o, ctx=ctx())
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    Wg, Hg, dg = Wd.cpu().numpy(), Hd.cpu().numpy(), o.item()
    del Vd, Wd, Hd
    V64, W64, H64 = p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64)
    d0 = O.objective(V64, W64, H64, p.beta)
    step = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    Wr, Hr = step(V64, W64, H64, p.beta)
    check_pair(Wg, Hg, Wr, Hr, precision, p.beta, tag=f"counts {mode} {precision}")
    if precision == "fp32":
        assert abs(dg - d0) <= 1e-6 * abs(d0), f"objective {dg} vs {d0}"
    else:
        tol = max(1e-6 * abs(d0), lowp_obj_bound(V64, W64, H64, p.beta))
        assert abs(dg - d0) <= tol, f"objective err {abs(dg - d0):.3e} > {tol:.3e}"


@pytest.mark.timeout(600)
def test_count_workload_full_size_objective_and_gradient(counts):
    # the objective-only and gradient passes at the size where V is streamed
    p = counts
    print(f"[fullsize] counts_kl objective and gradient F={p.V.shape[0]} N={p.V.shape[1]}", flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    d = nb.objective(Vd, Wd, Hd, p.beta, ctx=ctx()).item()
    dW, dH = nb.grad(Vd, Wd, Hd, p.beta, scale=1.0, ctx=ctx())
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    dW, dH = dW.cpu().numpy(), dH.cpu().numpy()
    del Vd, Wd, Hd
    V64, W64, H64 = p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64)
    d0 = O.objective(V64, W64, H64, p.beta)
    assert abs(d - d0) <= 1e-6 * abs(d0), (d, d0)
    gW, gH = O.gradient(V64, W64, H64, p.beta)
    # condition-scaled gates (E = Lambda^(beta-2) (Lambda - V) changes sign), as for the small shapes
    L = W64 @ H64
    E = np.abs(L ** (p.beta - 2) * (L - V64))
    sW, sH = np.linalg.norm(E @ np.abs(H64.T)), np.linalg.norm(np.abs(W64.T) @ E)
    assert np.linalg.norm(dW - gW) <= 1e-5 * sW
    assert np.linalg.norm(dH - gH) <= 1e-5 * sH


@pytest.fixture(scope="module")
def batched_full():
    """The 512 problems and the oracle's joint step of each (computed once)."""
    host, ref = [], []
    for i, sp in enumerate(synth.batched_specs()):
        if i % 64 == 0:
            print(f"[fullsize] oracle steps of the batched workload: problem {i}", flush=True)
        q = synth.make_batched_problem(sp)
        host.append((q.V, q.W, q.H, q.beta))
        V64, W64, H64 = q.V.astype(np.float64), q.W.astype(np.float64), q.H.astype(np.float64)
        ref.append(O.jmm_iteration(V64, W64, H64, q.beta) + (O.objective(V64, W64, H64, q.beta),))
    return host, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("tiles", [0, 128])
def test_batched_workload_full_size_all_problems(batched_full, tiles):
    host, ref = batched_full
    print(f"[fullsize] batched {len(host)} problems tiles_per_item={tiles}", flush=True)
    d = [(dev(V), dev(W), dev(H), b) for V, W, H, b in host]
    b = nb.Batch(d, "joint", tiles_per_item=tiles, ctx=ctx())
    print(f"[fullsize] batched {b.info()}", flush=True)
    obj = torch.full((len(d),), float("nan"), dtype=torch.float64, device=DEV)
    b.step(objectives=obj)
    torch.cuda.synchronize()
    assert b.flags() == 0
    b.close()
    ob = obj.cpu().numpy()
    assert np.all(np.isfinite(ob))
    worst = [0.0, 0.0]
    for i, ((V, W, H, beta), (Wr, Hr, d0)) in enumerate(zip(host, ref)):
        assert W.shape[1] < min(V.shape)  # no exact fit: the next iterate is unique
        (fw, ew), (fh, eh) = check_pair(d[i][1].cpu().numpy(), d[i][2].cpu().numpy(), Wr, Hr,
                                        tag=f"problem {i} {V.shape} K={W.shape[1]} beta={beta}")
        worst = [max(worst[0], fw, fh), max(worst[1], ew, eh)]
        assert abs(ob[i] - d0) <= 1e-6 * abs(d0), (i, ob[i], d0)
    print(f"[fullsize] batched worst Frobenius {worst[0]:.2e}, entry-wise {worst[1]:.2e}", flush=True)


@pytest.fixture(scope="module")
def above_pq_limit():
    F, N, K = 16449, 16353, 10
    assert F * N > 2 ** 28
    return synth.random_positive(F, N, K, seed=2028)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_joint_step_above_kept_pq_limit(above_pq_limit, precision):
    p = above_pq_limit
    beta = 0.5
    F, N = p.V.shape
    print(f"[fullsize] above the kept P/Q limit F={F} N={N} K={p.W.shape[1]} beta={beta} precision={precision}",
          flush=True)
    Vd, Wd, Hd = dev(p.V), dev(p.W), dev(p.H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    nb.step(Vd, Wd, Hd, beta, "joint", precision=precision, objective_out=o, ctx=ctx())
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    Wg, Hg, dg = Wd.cpu().numpy(), Hd.cpu().numpy(), o.item()
    del Vd, Wd, Hd
    V64, W64, H64 = p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64)
    d0 = O.objective(V64, W64, H64, beta)
    Wr, Hr = O.jmm_iteration(V64, W64, H64, beta)
    check_pair(Wg, Hg, Wr, Hr, precision, beta, tag=f"above P/Q limit {precision}")
    otol = 1e-6 * abs(d0) if precision == "fp32" else max(1e-6 * abs(d0), lowp_obj_bound(V64, W64, H64, beta))
    assert abs(dg - d0) <= otol, f"objective err {abs(dg - d0):.3e} > {otol:.3e}"
