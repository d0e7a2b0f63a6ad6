"""Pins for the oracle's beta = 1 iteration on a sparse V (CSR form).

The sparse forms must equal the dense oracle (itself pinned to the closed forms
of Table 2, the auxiliary function and finite differences) on the same data:
the objective, and one outer iteration of both methods, with and without
normalization, including rows and columns of V without any nonzero.  The
CSR conversion is checked against the dense matrix entry by entry.
"""
import numpy as np
import pytest

import oracle as O
import synth


def _case(seed, F=37, N=53, K=5, zeros=0.85, empty_row=True):
    p = synth.random_positive(F, N, K, seed=seed, zeros=zeros)
    V = p.V.copy()
    if empty_row:
        V[3, :] = 0.0   # an empty row
    V[:, 7] = 0.0   # an empty column
    return V, p.W.astype(np.float64), p.H.astype(np.float64)


def test_csr_and_csc_round_trip():
    V, _, _ = _case(0)
    rp, ci, v = synth.to_csr(V)
    D = np.zeros_like(V)
    for f in range(V.shape[0]):
        D[f, ci[rp[f]:rp[f + 1]]] = v[rp[f]:rp[f + 1]]
        assert np.all(np.diff(ci[rp[f]:rp[f + 1]]) > 0)
    assert np.array_equal(D, V) and rp[-1] == np.count_nonzero(V)
    cp, ri, w = synth.to_csc(V)
    E = np.zeros_like(V)
    for n in range(V.shape[1]):
        E[ri[cp[n]:cp[n + 1]], n] = w[cp[n]:cp[n + 1]]
    assert np.array_equal(E, V)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("zeros", [0.0, 0.5, 0.95])
def test_sparse_objective_equals_dense(seed, zeros):
    V, W, H = _case(seed, zeros=zeros)
    rp, ci, v = synth.to_csr(V)
    a = O.kl_sparse_objective(rp, ci, v, W, H)
    b = O.objective(V.astype(np.float64), W, H, 1.0)
    assert a == pytest.approx(b, rel=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("norm", [True, False])
def test_sparse_iteration_equals_dense(seed, mode, norm):
    # an empty row of V makes the row of W_new zero; in the alternating H step
    # the dense form then meets 0/0 at that row's (zero) entries, which the
    # sparse form never evaluates, so the dense comparison uses a V without one
    V, W, H = _case(seed, empty_row=(mode == "joint"))
    rp, ci, v = synth.to_csr(V)
    Ws, Hs = O.kl_sparse_iteration(rp, ci, v, W, H, mode, norm=norm)
    dense = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    Wd, Hd = dense(V.astype(np.float64), W, H, 1.0, norm=norm)
    assert np.allclose(Ws, Wd, rtol=1e-12, atol=0) and np.allclose(Hs, Hd, rtol=1e-12, atol=0)
    # an empty column of V gives a zero column of H_new (and an empty row a zero row of W_new)
    assert np.all(Hs[:, 7] == 0)
    if mode == "joint":
        assert np.all(Ws[3] == 0)


@pytest.mark.parametrize("norm", [True, False])
def test_sparse_alternating_with_an_empty_row_equals_dense_without_it(norm):
    # Row 3 of V is empty: W_new[3] = 0 and the row adds nothing to the H step's
    # numerator (no nonzeros) or denominator (a zero row of W_new), so the
    # result equals the dense iteration on V, W without row 3, with W_new[3] = 0.
    V, W, H = _case(4)
    rp, ci, v = synth.to_csr(V)
    Ws, Hs = O.kl_sparse_iteration(rp, ci, v, W, H, "alternating", norm=norm)
    keep = np.arange(V.shape[0]) != 3
    Wd, Hd = O.bmm_iteration(V[keep].astype(np.float64), W[keep], H, 1.0, norm=norm)
    assert np.all(Ws[3] == 0)
    assert np.allclose(Ws[keep], Wd, rtol=1e-12, atol=0) and np.allclose(Hs, Hd, rtol=1e-12, atol=0)


def test_sparse_iterations_decrease_the_objective():
    V, W, H = _case(9, F=60, N=70, K=4, zeros=0.9)
    V[3, :] = 1.0  # keep every row and column populated for a multi-step run
    V[:, 7] = 1.0
    rp, ci, v = synth.to_csr(V)
    for mode in ("joint", "alternating"):
        Wm, Hm = W.copy(), H.copy()
        d = [O.kl_sparse_objective(rp, ci, v, Wm, Hm)]
        for _ in range(30):
            Wm, Hm = O.kl_sparse_iteration(rp, ci, v, Wm, Hm, mode)
            d.append(O.kl_sparse_objective(rp, ci, v, Wm, Hm))
        assert np.all(np.diff(d) <= 1e-12 * np.abs(d[1:]))


def test_count_workload_crop_density():
    # the two count workloads: about 8.5 % and about 1 % nonzeros (a 512-row block)
    a = synth.make_problem("counts_kl", rows=(0, 512))
    b = synth.make_problem("counts_kl_sparse", rows=(0, 512))
    da, db = np.count_nonzero(a.V) / a.V.size, np.count_nonzero(b.V) / b.V.size
    assert 0.07 < da < 0.10 and 0.006 < db < 0.015, (da, db)
