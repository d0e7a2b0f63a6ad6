"""GPU parity of the beta = 1 step on a sparse V (nmf_kl_step_sparse) against the
FP64 oracle's sparse iteration (itself pinned to the dense oracle).

Gates (tests/gates.py): W, H relative Frobenius error <= 1e-5 and entry-wise
<= 1e-4 (float32 arithmetic: lambda is a K-term dot product, the numerators
sums over a row's or column's nonzeros, the denominators float64 sums);
objective <= 1e-6 relative.  Cases: ragged shapes and ranks K in 1..64,
densities from 0.5 % to 100 %, empty rows and columns, both methods, with and
without normalization, crops of both count workloads, and both count workloads
at full size (20000 x 10000, K = 50, about 1 % and 8.5 % nonzeros).
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


def sparse_dev(V):
    rp, ci, rv = synth.to_csr(V)
    cp, ri, cv = synth.to_csc(V)
    return nb.SparseV(V.shape[0], V.shape[1], dev(rp), dev(ci), dev(rv), dev(cp), dev(ri), dev(cv))


def check_sparse_step(V, W, H, mode, normalize=True, tag=""):
    F, N = V.shape
    K = W.shape[1]
    print(f"[sparse] {tag} F={F} N={N} K={K} nnz={np.count_nonzero(V)} mode={mode} norm={normalize}", flush=True)
    Vs = sparse_dev(V)
    Wd, Hd = dev(W), dev(H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    nb.kl_step_sparse(Vs, Wd, Hd, mode, normalize=normalize, objective_out=o, ctx=ctx())
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    rp, ci, rv = synth.to_csr(V)
    W64, H64 = W.astype(np.float64), H.astype(np.float64)
    Wr, Hr = O.kl_sparse_iteration(rp, ci, rv, W64, H64, mode, norm=normalize)
    check_pair(Wd.cpu().numpy(), Hd.cpu().numpy(), Wr, Hr, tag=tag)
    d0 = O.kl_sparse_objective(rp, ci, rv, W64, H64)
    assert abs(o.item() - d0) <= 1e-6 * abs(d0), (o.item(), d0)
    return Wd, Hd


SHAPES = [(64, 100, 5), (200, 150, 20), (257, 300, 49), (130, 70, 64), (33, 1000, 8), (1, 40, 3), (40, 1, 3),
          (129, 129, 1), (96, 160, 32), (500, 77, 17)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("zeros", [0.0, 0.7, 0.97])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_sparse_step_parity_shapes(shape, zeros, mode):
    F, N, K = shape
    p = synth.random_positive(F, N, K, seed=F * 3 + N + K, zeros=zeros)
    V = p.V.copy()
    if F > 3 and N > 3 and mode == "joint":
        V[2, :] = 0.0   # an empty row
    if N > 5:
        V[:, 4] = 0.0   # an empty column
    check_sparse_step(V, p.W, p.H, mode, tag=f"shape zeros={zeros}")


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_sparse_step_without_normalization(mode):
    p = synth.random_positive(180, 210, 12, seed=5, zeros=0.9)
    check_sparse_step(p.V, p.W, p.H, mode, normalize=False, tag="nonorm")


@pytest.mark.parametrize("name", ["counts_kl", "counts_kl_sparse"])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_sparse_step_count_crops(name, mode):
    p = synth.make_problem(name, rows=(1000, 1700), cols=(3000, 4100))
    check_sparse_step(p.V, p.W, p.H, mode, tag=name)


@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_sparse_trajectory_monotone_and_matches_dense_gpu(mode):
    # 30 iterations: the objective decreases at every step, and the sparse and
    # dense GPU paths follow the same trajectory.  A crop of the 8.5 % count
    # workload: every row and column has nonzeros (an empty row would make the
    # dense path's V / (WH) the undefined 0/0 once its row of W is zero).
    p = synth.make_problem("counts_kl", rows=(0, 600), cols=(0, 900))
    assert np.all(np.any(p.V != 0, axis=0)) and np.all(np.any(p.V != 0, axis=1))
    Vs = sparse_dev(p.V)
    Vd = dev(p.V)
    Ws, Hs = dev(p.W), dev(p.H)
    Wd, Hd = dev(p.W), dev(p.H)
    o = torch.zeros(1, dtype=torch.float64, device=DEV)
    trace = []
    for _ in range(30):
        nb.kl_step_sparse(Vs, Ws, Hs, mode, objective_out=o, ctx=ctx())
        trace.append(o.item())
        nb.step(Vd, Wd, Hd, 1.0, mode, ctx=ctx())
    torch.cuda.synchronize()
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    trace = np.array(trace)
    assert np.all(trace[1:] <= trace[:-1] * (1 + 4e-7)), np.max(np.diff(trace) / trace[:-1])
    check_pair(Ws.cpu().numpy(), Hs.cpu().numpy(), Wd.cpu().numpy(), Hd.cpu().numpy(), tag="sparse vs dense GPU",
               fro=3e-5, el=3e-4)


def test_sparse_objective_call_and_from_dense():
    p = synth.random_positive(300, 411, 25, seed=7, zeros=0.95)
    V = p.V
    Vs = nb.SparseV.from_dense(dev(V))
    Vh = sparse_dev(V)
    for a, b in ((Vs.row_ptr, Vh.row_ptr), (Vs.col_idx, Vh.col_idx), (Vs.row_val, Vh.row_val),
                 (Vs.col_ptr, Vh.col_ptr), (Vs.row_idx, Vh.row_idx), (Vs.col_val, Vh.col_val)):
        assert torch.equal(a, b)
    d = nb.kl_objective_sparse(Vs, dev(p.W), dev(p.H), ctx=ctx()).item()
    rp, ci, rv = synth.to_csr(V)
    d0 = O.kl_sparse_objective(rp, ci, rv, p.W.astype(np.float64), p.H.astype(np.float64))
    assert abs(d - d0) <= 1e-6 * abs(d0)
    dd = nb.objective(dev(V), dev(p.W), dev(p.H), 1.0, ctx=ctx()).item()
    assert abs(d - dd) <= 1e-6 * abs(d0)


def test_sparse_validate_and_rejections():
    p = synth.random_positive(50, 60, 6, seed=8, zeros=0.8)
    Vs = sparse_dev(p.V)
    nb.sparse_validate(Vs, ctx=ctx())
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    bad = sparse_dev(p.V)
    bad.col_idx[3] = 60  # out of range: flagged; a step reads it clamped (no fault)
    nb.sparse_validate(bad, ctx=ctx())
    assert nb.get_flags(clear=True, ctx=ctx()) & nb.FLAG_DOMAIN
    neg = sparse_dev(p.V)
    neg.row_val[0] = -1.0
    nb.sparse_validate(neg, ctx=ctx())
    assert nb.get_flags(clear=True, ctx=ctx()) & nb.FLAG_DOMAIN
    W, H = dev(p.W), dev(p.H)
    with pytest.raises(nb.NmfError):  # K > 64
        q = synth.random_positive(50, 60, 65, seed=9)
        nb.kl_step_sparse(Vs, dev(q.W), dev(q.H), "joint", ctx=ctx())
    L = nb.lib()
    o = nb._opts(kappa=0.1)
    sv = Vs._struct()
    import ctypes
    assert L.nmf_kl_step_sparse(ctx().handle, None, ctypes.byref(sv), 6, W.data_ptr(), 6, H.data_ptr(), 60, 1,
                                ctypes.byref(o), None) == 7  # kappa > 0: unsupported
    assert torch.equal(W, dev(p.W))


@pytest.fixture(scope="module", params=["counts_kl_sparse", "counts_kl"])
def counts_full(request):
    p = synth.make_problem(request.param)
    rp, ci, rv = synth.to_csr(p.V)
    return p, (rp, ci, rv)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["joint", "alternating"])
def test_sparse_count_workload_full_size(counts_full, mode):
    p, (rp, ci, rv) = counts_full
    W64, H64 = p.W.astype(np.float64), p.H.astype(np.float64)
    check_sparse_step(p.V, p.W, p.H, mode, tag=f"full {p.name}")
