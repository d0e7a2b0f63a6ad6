"""Pins for the FP64 CPU oracle: checks against what the paper and mathematics fix.

None of these re-types the oracle's own formula.  They use closed forms
(fixture file), brute-force pure-Python loops, exact rational arithmetic on the
textbook / simplified update forms of Table 2 (Sec. 3.3.1), the joint auxiliary
function of Sec. 3.1 (tightness, majorization, stationarity of the updates,
descent chain), finite differences, invariants (monotone decrease of the MM
objective, positivity, scale equivariance, fixed points) and library routines.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
BETAS = [-0.5, 0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0]


def _small(seed=0, F=6, N=7, K=3, zeros=0.0):
    p = synth.random_positive(F, N, K, seed=seed, zeros=zeros)
    return p.V.astype(np.float64), p.W.astype(np.float64), p.H.astype(np.float64)


# ---------------------------------------------------------------------------
# beta-divergence, eq. (beta-div)
# ---------------------------------------------------------------------------
def _golden_points():
    rows = []
    with open(os.path.join(GOLD, "d_beta_points.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append(tuple(float(t) for t in line.split()))
    return rows


@pytest.mark.parametrize("beta,x,y,val", _golden_points())
def test_d_beta_closed_forms(beta, x, y, val):
    got = float(O.beta_divergence(x, y, beta))
    assert got == pytest.approx(val, rel=1e-14, abs=1e-15)


@pytest.mark.parametrize("b0,eps", [(1.0, 1e-6), (1.0, -1e-6), (0.0, 1e-6), (0.0, -1e-6)])
def test_d_beta_continuous_in_beta(b0, eps):
    # the general branch tends to the KL / IS branches (eq. beta-div)
    x = np.array([0.3, 1.0, 2.0, 7.5])
    y = np.array([1.1, 0.4, 2.0, 3.0])
    lim = O.beta_divergence(x, y, b0)
    near = O.beta_divergence(x, y, b0 + eps)
    # O(eps) true deviation plus O(1e-16/eps) cancellation in the general branch
    assert np.allclose(near, lim, rtol=2e-5, atol=1e-7)


@pytest.mark.parametrize("beta", BETAS)
def test_d_beta_homogeneity_and_positivity(beta):
    rng = np.random.default_rng(3)
    x = rng.uniform(0.1, 5, 50)
    y = rng.uniform(0.1, 5, 50)
    c = 2.7
    d = O.beta_divergence(x, y, beta)
    assert np.all(d >= -1e-14)
    assert np.allclose(O.beta_divergence(c * x, c * y, beta), c ** beta * d, rtol=1e-11, atol=1e-13)
    assert np.allclose(O.beta_divergence(x, x, beta), 0.0, atol=1e-12)


def test_objective_beta2_is_half_frobenius():
    V, W, H = _small(1, 9, 11, 4)
    ref = 0.5 * np.linalg.norm(V - W @ H, "fro") ** 2
    assert O.objective(V, W, H, 2.0) == pytest.approx(ref, rel=1e-13)


def _brute_objective(V, W, H, beta, kappa=0.0):
    F, K = len(W), len(W[0])
    N = len(H[0])
    tot = 0.0
    for f in range(F):
        for n in range(N):
            y = kappa
            for k in range(K):
                y += W[f][k] * H[k][n]
            x = V[f][n] + kappa
            if beta == 1.0:
                d = (x * math.log(x / y) if x > 0 else 0.0) - x + y
            elif beta == 0.0:
                d = x / y - math.log(x / y) - 1.0
            else:
                d = x ** beta / (beta * (beta - 1)) + y ** beta / beta - x * y ** (beta - 1) / (beta - 1)
            tot += d
    return tot


@pytest.mark.parametrize("beta", BETAS)
def test_objective_brute_force(beta):
    zeros = 0.2 if beta > 0 else 0.0
    V, W, H = _small(2, 5, 8, 3, zeros=zeros)
    got = O.objective(V, W, H, beta)
    ref = _brute_objective(V.tolist(), W.tolist(), H.tolist(), beta)
    assert got == pytest.approx(ref, rel=1e-12)


def test_objective_kappa_shift():
    V, W, H = _small(4, 5, 6, 2, zeros=0.3)
    kap = 0.05
    ref = _brute_objective(V.tolist(), W.tolist(), H.tolist(), 0.0, kappa=kap)
    assert O.objective(V, W, H, 0.0, kappa=kap) == pytest.approx(ref, rel=1e-12)


def test_gamma_exponent_values():
    assert O.gamma_exponent(0.0) == 0.5
    assert O.gamma_exponent(0.5) == pytest.approx(1 / 1.5)
    assert O.gamma_exponent(-1.0) == pytest.approx(1 / 3)
    for b in (1.0, 1.2, 2.0):
        assert O.gamma_exponent(b) == 1.0
    assert O.gamma_exponent(3.0) == 0.5


# ---------------------------------------------------------------------------
# update rules against exact rational Table-2 / textbook forms (beta = 1, 2)
# ---------------------------------------------------------------------------
def _F(a):
    return [[Fraction(float(v)) for v in row] for row in np.atleast_2d(a)]


def _mm(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))] for i in range(len(A))]


def _T(A):
    return [list(r) for r in zip(*A)]


def _ew(f, *Ms):
    return [[f(*vals) for vals in zip(*rows)] for rows in zip(*Ms)]


def _ones(r, c):
    return [[Fraction(1)] * c for _ in range(r)]


def _exact_steps(V, Wt, Ht, beta):
    """Exact W step (shared by both methods at L=1) and both H steps.

    beta = 2: Lee-Seung W <- W (V H^T)/(W H H^T); BMM H <- H (W^T V)/(W^T W H);
              JMM H <- H~ (W^T V)/((W^2/W~)^T W~ H~)          (Table 2, beta = 2)
    beta = 1: W <- W ((V/WH) H^T)/(1 H^T); BMM H <- H (W^T (V/WH))/(W^T 1);
              JMM H <- H~ (W~^T (V/W~H~))/(W^T 1)              (Table 2, beta = 1)
    """
    Vq, Wq, Hq = _F(V), _F(Wt), _F(Ht)
    F_, N_ = len(Vq), len(Vq[0])
    Lt = _mm(Wq, Hq)
    if beta == 2.0:
        Wn = _ew(lambda w, a, b: w * a / b, Wq, _mm(Vq, _T(Hq)), _mm(Lt, _T(Hq)))
        L2 = _mm(Wn, Hq)
        Hb = _ew(lambda h, a, b: h * a / b, Hq, _mm(_T(Wn), Vq), _mm(_T(Wn), L2))
        chi = _ew(lambda w, wt: w * w / wt, Wn, Wq)
        Hj = _ew(lambda h, a, b: h * a / b, Hq, _mm(_T(Wn), Vq), _mm(_T(chi), Lt))
    else:
        R = _ew(lambda v, l: v / l, Vq, Lt)
        Wn = _ew(lambda w, a, b: w * a / b, Wq, _mm(R, _T(Hq)), _mm(_ones(F_, N_), _T(Hq)))
        R2 = _ew(lambda v, l: v / l, Vq, _mm(Wn, Hq))
        Hb = _ew(lambda h, a, b: h * a / b, Hq, _mm(_T(Wn), R2), _mm(_T(Wn), _ones(F_, N_)))
        Hj = _ew(lambda h, a, b: h * a / b, Hq, _mm(_T(Wq), R), _mm(_T(Wn), _ones(F_, N_)))
    tofl = lambda M: np.array([[float(v) for v in r] for r in M])
    return tofl(Wn), tofl(Hb), tofl(Hj)


@pytest.mark.parametrize("beta", [1.0, 2.0])
@pytest.mark.parametrize("seed", [0, 1])
def test_updates_match_exact_table2(beta, seed):
    V, W, H = _small(seed, 4, 5, 2)
    Wn, Hb, Hj = _exact_steps(V, W, H, beta)
    Wb_o, Hb_o = O.bmm_iteration(V, W, H, beta, norm=False)
    Wj_o, Hj_o = O.jmm_iteration(V, W, H, beta, norm=False)
    assert np.allclose(Wb_o, Wn, rtol=1e-13, atol=0)
    assert np.allclose(Wj_o, Wn, rtol=1e-13, atol=0)
    assert np.allclose(Hb_o, Hb, rtol=1e-13, atol=0)
    assert np.allclose(Hj_o, Hj, rtol=1e-13, atol=0)
    # the two H updates really differ (a pin that cannot pass by accident)
    assert not np.allclose(Hb, Hj, rtol=1e-6)


def _loop_mm(A, B):
    A = np.asarray(A)
    B = np.asarray(B)
    out = np.zeros((A.shape[0], B.shape[1]))
    for i in range(A.shape[0]):
        for j in range(B.shape[1]):
            s = 0.0
            for k in range(A.shape[1]):
                s += A[i, k] * B[k, j]
            out[i, j] = s
    return out


@pytest.mark.parametrize("seed", [0, 3])
def test_is_updates_match_table2_beta0(seed):
    # Table 2, beta = 0 (gamma = 1/2), loops in float64:
    #   BMM:  H <- H ((W^T (V/(WH)^2)) / (W^T (1/WH)))^(1/2)
    #   JMM:  H <- H~ (((W~^2/W)^T (V/(W~H~)^2)) / (W^T (1/(W~H~))))^(1/2)
    # and the shared W step W <- W~ (((V/(W~H~)^2) H~^T) / ((1/W~H~) H~^T))^(1/2).
    V, Wt, Ht = _small(seed, 5, 6, 3)
    Lt = _loop_mm(Wt, Ht)
    Wn = Wt * np.sqrt(_loop_mm(V / Lt ** 2, Ht.T) / _loop_mm(1.0 / Lt, Ht.T))
    L2 = _loop_mm(Wn, Ht)
    Hb = Ht * np.sqrt(_loop_mm(Wn.T, V / L2 ** 2) / _loop_mm(Wn.T, 1.0 / L2))
    Hj = Ht * np.sqrt(_loop_mm((Wt ** 2 / Wn).T, V / Lt ** 2) / _loop_mm(Wn.T, 1.0 / Lt))
    Wb_o, Hb_o = O.bmm_iteration(V, Wt, Ht, 0.0, norm=False)
    Wj_o, Hj_o = O.jmm_iteration(V, Wt, Ht, 0.0, norm=False)
    assert np.allclose(Wb_o, Wn, rtol=1e-13)
    assert np.allclose(Wj_o, Wn, rtol=1e-13)
    assert np.allclose(Hb_o, Hb, rtol=1e-13)
    assert np.allclose(Hj_o, Hj, rtol=1e-13)


# ---------------------------------------------------------------------------
# joint auxiliary function G (Sec. 3.1): tightness, majorization, stationarity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beta", BETAS)
def test_G_tight_and_majorizes(beta):
    V, Wt, Ht = _small(5, 6, 7, 3)
    D0 = O.objective(V, Wt, Ht, beta)
    assert O.joint_auxiliary(V, Wt, Ht, Wt, Ht, beta) == pytest.approx(D0, rel=1e-13)
    rng = np.random.default_rng(11)
    for _ in range(30):
        W = Wt * rng.uniform(0.3, 3.0, Wt.shape)
        H = Ht * rng.uniform(0.3, 3.0, Ht.shape)
        G = O.joint_auxiliary(V, W, H, Wt, Ht, beta)
        D = O.objective(V, W, H, beta)
        assert G >= D - 1e-12 * abs(D)


def _num_grad(fun, X, h=1e-6):
    g = np.zeros_like(X)
    for idx in np.ndindex(X.shape):
        e = np.zeros_like(X)
        step = h * max(1.0, abs(X[idx]))
        e[idx] = step
        g[idx] = (fun(X + e) - fun(X - e)) / (2 * step)
    return g


@pytest.mark.parametrize("beta", BETAS)
def test_jmm_updates_are_stationary_points_of_G(beta):
    # eq. (jnt_update) cancels the partial gradients of G (Sec. 3.2):
    # W_new minimizes G(., H~ | W~, H~), then H_new minimizes G(W_new, . | W~, H~).
    V, Wt, Ht = _small(6, 5, 6, 3)
    _, _, parts = O.jmm_iteration(V, Wt, Ht, beta, norm=False, return_parts=True)
    Wn, Hn = parts["W_unnorm"], parts["H_unnorm"]
    gW = _num_grad(lambda W: O.joint_auxiliary(V, W, Ht, Wt, Ht, beta), Wn)
    gH = _num_grad(lambda H: O.joint_auxiliary(V, Wn, H, Wt, Ht, beta), Hn)
    scale = O.objective(V, Wt, Ht, beta)
    assert np.max(np.abs(gW)) < 1e-6 * scale
    assert np.max(np.abs(gH)) < 1e-6 * scale


@pytest.mark.parametrize("beta", BETAS)
def test_bmm_updates_are_stationary_points_of_blockwise_G(beta):
    # BMM (L=1) written with the same G (Sec. 3.3.3): the H update minimizes
    # G(W_new, . | W_new, H~), i.e. tilde-W is replaced by the new W.
    V, Wt, Ht = _small(7, 5, 6, 3)
    _, _, parts = O.bmm_iteration(V, Wt, Ht, beta, norm=False, return_parts=True)
    Wn, Hn = parts["W_unnorm"], parts["H_unnorm"]
    gW = _num_grad(lambda W: O.joint_auxiliary(V, W, Ht, Wt, Ht, beta), Wn)
    gH = _num_grad(lambda H: O.joint_auxiliary(V, Wn, H, Wn, Ht, beta), Hn)
    scale = O.objective(V, Wt, Ht, beta)
    assert np.max(np.abs(gW)) < 1e-6 * scale
    assert np.max(np.abs(gH)) < 1e-6 * scale


@pytest.mark.parametrize("beta", BETAS)
def test_jmm_descent_chain(beta):
    # D(W_new H_new) <= G(W_new,H_new) <= G(W_new,H~) <= G(W~,H~) = D(W~H~)  (descent lemma)
    V, Wt, Ht = _small(8, 6, 7, 3)
    _, _, parts = O.jmm_iteration(V, Wt, Ht, beta, norm=False, return_parts=True)
    Wn, Hn = parts["W_unnorm"], parts["H_unnorm"]
    tol = 1e-12
    d1 = O.objective(V, Wn, Hn, beta)
    g1 = O.joint_auxiliary(V, Wn, Hn, Wt, Ht, beta)
    g2 = O.joint_auxiliary(V, Wn, Ht, Wt, Ht, beta)
    g3 = O.joint_auxiliary(V, Wt, Ht, Wt, Ht, beta)
    d0 = O.objective(V, Wt, Ht, beta)
    assert d1 <= g1 * (1 + tol) and g1 <= g2 * (1 + tol) and g2 <= g3 * (1 + tol)
    assert g3 == pytest.approx(d0, rel=1e-13)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("mode", ["bmm", "jmm"])
@pytest.mark.parametrize("L", [1, 3])
def test_monotone_decrease_and_positivity(beta, mode, L):
    V, W, H = _small(9, 12, 15, 4)
    D = [O.objective(V, W, H, beta)]
    for _ in range(120):
        if mode == "bmm":
            W, H = O.bmm_iteration(V, W, H, beta, L_W=L, L_H=L)
        else:
            W, H = O.jmm_iteration(V, W, H, beta, L=L)
        D.append(O.objective(V, W, H, beta))
        assert W.min() > 0 and H.min() > 0
    D = np.array(D)
    assert np.all(np.diff(D) <= 1e-13 * D[:-1])
    assert D[-1] < 0.9 * D[0]


@pytest.mark.parametrize("beta", BETAS)
def test_w_steps_coincide_at_L1(beta):
    V, W, H = _small(10, 7, 9, 3)
    Wb, _ = O.bmm_iteration(V, W, H, beta, norm=False)
    Wj, _ = O.jmm_iteration(V, W, H, beta, norm=False)
    assert np.allclose(Wb, Wj, rtol=1e-14, atol=0)


@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5, 2.0])
@pytest.mark.parametrize("mode", ["bmm", "jmm"])
def test_exact_factorization_is_fixed_point(beta, mode):
    rng = np.random.default_rng(12)
    W0 = rng.uniform(0.5, 2, (6, 2))
    H0 = rng.uniform(0.5, 2, (2, 8))
    V = W0 @ H0
    f = O.bmm_iteration if mode == "bmm" else O.jmm_iteration
    W1, H1 = f(V, W0, H0, beta, norm=False)
    assert np.allclose(W1, W0, rtol=1e-13) and np.allclose(H1, H0, rtol=1e-13)
    assert O.objective(V, W0, H0, beta) == pytest.approx(0.0, abs=1e-12)
    rW, rH = O.kkt_residuals(V, W0, H0, beta)
    assert rW < 1e-13 and rH < 1e-13


def test_normalize_unit_columns_product_unchanged():
    V, W, H = _small(13, 8, 9, 3)
    W[:, 1] = 0.0
    Wn, Hn = O.normalize(W, H)
    norms = np.linalg.norm(Wn, axis=0)
    assert np.allclose(norms[[0, 2]], 1.0, rtol=1e-15)
    assert np.all(Wn[:, 1] == 0.0) and np.all(Hn[1] == H[1])
    assert np.allclose(Wn @ Hn, W @ H, rtol=1e-14)


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("mode", ["bmm", "jmm"])
def test_normalization_does_not_change_trajectory(beta, mode):
    # both updates are scale-equivariant, so normalizing only rescales the factors
    V, W, H = _small(14, 6, 8, 3)
    f = O.bmm_iteration if mode == "bmm" else O.jmm_iteration
    Wa, Ha = W, H
    Wb, Hb = W, H
    for _ in range(5):
        Wa, Ha = f(V, Wa, Ha, beta, norm=True)
        Wb, Hb = f(V, Wb, Hb, beta, norm=False)
    assert np.allclose(Wa @ Ha, Wb @ Hb, rtol=1e-11)


@pytest.mark.parametrize("beta", BETAS)
def test_gradient_finite_differences(beta):
    V, W, H = _small(15, 5, 6, 3)
    gW, gH = O.gradient(V, W, H, beta)
    nW = _num_grad(lambda X: O.objective(V, X, H, beta), W)
    nH = _num_grad(lambda X: O.objective(V, W, X, beta), H)
    assert np.allclose(gW, nW, rtol=1e-6, atol=1e-8 * np.abs(nW).max())
    assert np.allclose(gH, nH, rtol=1e-6, atol=1e-8 * np.abs(nH).max())


@pytest.mark.parametrize("beta", BETAS)
def test_gradient_is_den_minus_num(beta):
    # numerator / denominator of the multiplicative updates are the negative /
    # positive parts of the gradient at the point where they are evaluated
    V, W, H = _small(16, 5, 6, 3)
    _, _, parts = O.bmm_iteration(V, W, H, beta, norm=False, return_parts=True)
    gW, _ = O.gradient(V, W, H, beta)
    assert np.allclose(parts["denW"] - parts["numW"], gW, rtol=1e-10, atol=1e-12)
    _, gH = O.gradient(V, parts["W_unnorm"], H, beta)
    assert np.allclose(parts["denH"] - parts["numH"], gH, rtol=1e-10, atol=1e-12)


def test_nonfinite_ratio_raises():
    V, W, H = _small(17, 4, 5, 2)
    H[:, :] = 0.0
    with pytest.raises(FloatingPointError):
        O.jmm_iteration(V, W, H, 1.0)


def test_kappa_allows_zeros_for_is():
    V, W, H = _small(18, 6, 7, 3, zeros=0.3)
    D = [O.objective(V, W, H, 0.0, kappa=1e-2)]
    for _ in range(30):
        W, H = O.jmm_iteration(V, W, H, 0.0, kappa=1e-2)
        D.append(O.objective(V, W, H, 0.0, kappa=1e-2))
    assert np.all(np.isfinite(D)) and np.all(np.diff(D) <= 1e-12 * np.array(D[:-1]))


def test_jmm_L_greater_than_one_keeps_tilde_base():
    # Algorithm 2: every sub-iteration multiplies W~ and H~; with L=2 the second
    # W update uses chi(H_2, H~) in the ratio but W~ as the base.
    V, Wt, Ht = _small(19, 5, 6, 3)
    beta = 0.5
    g = O.gamma_exponent(beta)
    W2, H2 = O.jmm_iteration(V, Wt, Ht, beta, L=2, norm=False)
    W1, H1 = O.jmm_iteration(V, Wt, Ht, beta, L=1, norm=False)
    Lt = Wt @ Ht
    P = V * Lt ** (beta - 2)
    Q = Lt ** (beta - 1)
    c1 = Ht ** (2 - beta) / H1 ** (1 - beta)
    Wexp = Wt * ((P @ c1.T) / (Q @ H1.T)) ** g
    assert np.allclose(W2, Wexp, rtol=1e-12)


# ---------------------------------------------------------------------------
# the heuristic exponent gamma = 1 (Sec. 3.3.3, "Failure of heuristic updates")
# ---------------------------------------------------------------------------
def test_heuristic_exponent_at_beta_zero_is_the_textbook_is_update():
    # block MM with gamma = 1 at beta = 0: the classical Itakura-Saito
    # multiplicative rules W <- W (V/L^2 H^T) / (1/L H^T), then H likewise against
    # the new W, written out here in plain matrix form
    V, W, H = _small(31, 8, 11, 3)
    L = W @ H
    W1 = W * (((V / L**2) @ H.T) / ((1.0 / L) @ H.T))
    L = W1 @ H
    H1 = H * ((W1.T @ (V / L**2)) / (W1.T @ (1.0 / L)))
    Wo, Ho = O.bmm_iteration(V, W, H, 0.0, norm=False, exponent="one")
    assert np.allclose(Wo, W1, rtol=1e-13, atol=0) and np.allclose(Ho, H1, rtol=1e-13, atol=0)


@pytest.mark.parametrize("beta", [1.0, 1.2, 1.5, 2.0])
@pytest.mark.parametrize("mode", ["bmm", "jmm"])
def test_heuristic_exponent_changes_nothing_where_gamma_is_one(beta, mode):
    # gamma(beta) = 1 on [1, 2] (eq. def_gamma), so both exponents give the same step
    V, W, H = _small(32, 7, 9, 3)
    f = O.bmm_iteration if mode == "bmm" else O.jmm_iteration
    Wa, Ha = f(V, W, H, beta)
    Wb, Hb = f(V, W, H, beta, exponent="one")
    assert np.array_equal(Wa, Wb) and np.array_equal(Ha, Hb)


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_heuristic_exponent_decreases_block_mm_objective_on_zero_one(beta):
    # for beta in [0, 1] the gamma = 1 block update is a majorization-equalization
    # scheme, which the paper cites as proven to decrease the objective
    V, W, H = _small(33, 12, 15, 4)
    D = [O.objective(V, W, H, beta)]
    for _ in range(100):
        W, H = O.bmm_iteration(V, W, H, beta, exponent="one")
        D.append(O.objective(V, W, H, beta))
    D = np.array(D)
    assert np.all(np.diff(D) <= 1e-13 * D[:-1])


@pytest.mark.parametrize("beta", [-0.5, 0.0, 0.5, 2.5])
def test_heuristic_exponent_w_steps_coincide_at_L1(beta):
    # at L = 1 the joint W step multiplies the same P H~^T / Q H~^T as block MM
    V, W, H = _small(34, 7, 9, 3)
    Wb, _ = O.bmm_iteration(V, W, H, beta, norm=False, exponent="one")
    Wj, _ = O.jmm_iteration(V, W, H, beta, norm=False, exponent="one")
    assert np.allclose(Wb, Wj, rtol=1e-14, atol=0)
    Wm, _ = O.bmm_iteration(V, W, H, beta, norm=False)
    assert not np.allclose(Wm, Wb, rtol=1e-6, atol=0)  # the exponent matters outside [1, 2]


# ---------------------------------------------------------------------------
# KKT residuals (Sec. 4.1.5) and the stopping rule (Sec. 4.1.2), against
# hand-evaluated fixtures
# ---------------------------------------------------------------------------
def _mat_field(text):
    return np.array([[float(t) for t in row.split()] for row in text.split(";")], dtype=np.float64)


def _kkt_cases():
    rows = []
    with open(os.path.join(GOLD, "kkt_residuals.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = [x.strip() for x in line.split("|")]
            rows.append((float(f[0]), _mat_field(f[1]), _mat_field(f[2]), _mat_field(f[3]), float(f[4]),
                         float(f[5])))
    return rows


@pytest.mark.parametrize("case", range(2))
def test_kkt_residuals_hand_cases(case):
    beta, V, W, H, rW, rH = _kkt_cases()[case]
    F, N = V.shape
    K = W.shape[1]
    assert len({F * K, K * N, F * N}) == 3 or K == 1  # normalizations distinguishable
    got = O.kkt_residuals(V, W, H, beta)
    assert got[0] == pytest.approx(rW, rel=1e-14)
    assert got[1] == pytest.approx(rH, rel=1e-14)


def test_kkt_residuals_zero_at_interior_stationary_point():
    # an exact factorization has zero gradient, and every W, H entry is > 0 so
    # min(X, 0) = 0: both residuals vanish (the KKT conditions hold)
    V, W, H = _small(seed=3)
    V = W @ H
    for beta in (0.0, 1.0, 2.0, 0.5):
        rW, rH = O.kkt_residuals(V, W, H, beta)
        assert rW < 1e-12 and rH < 1e-12


def test_kkt_residuals_boundary_point_with_positive_gradient():
    # W entry at 0 with a positive gradient component: min(0, g) = 0 there, so
    # the residual is not the gradient norm (complementarity, Sec. 4.1.5)
    V = np.array([[1.0, 2.0], [3.0, 4.0]])
    W = np.array([[0.0], [1.0]])
    H = np.array([[5.0, 5.0]])
    # beta = 2: E = WH - V = [[-1, -2], [2, 1]]; grad_W = E H^T = [[-15], [15]]
    # min(W, grad_W) = [[-15], [1]] -> 16 / (F K = 2) = 8
    # grad_H = W^T E = [[2, 1]]; min(H, grad_H) = [[2, 1]] -> 3 / (K N = 2) = 1.5
    rW, rH = O.kkt_residuals(V, W, H, 2.0)
    assert rW == pytest.approx(8.0, rel=1e-15)
    assert rH == pytest.approx(1.5, rel=1e-15)


def _stop_cases():
    rows = []
    with open(os.path.join(GOLD, "stop_rule.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = [x.strip() for x in line.split("|")]
            rows.append((float(f[0]), [float(t) for t in f[1].split()], None if f[2] == "none" else int(f[2])))
    return rows


@pytest.mark.parametrize("case", range(7))
def test_stop_rule_hand_cases(case):
    eps, trace, want = _stop_cases()[case]
    assert O.stop_iteration(trace, eps) == want


def test_relative_decrease_sign_convention():
    # positive for a decrease, negative for an increase, relative to the current value
    assert O.relative_decrease(2.0, 1.0) == 1.0
    assert O.relative_decrease(1.0, 2.0) == -0.5
    assert O.relative_decrease(3.0, 3.0) == 0.0
    assert O.relative_decrease(10.0, 8.0) == pytest.approx(0.25, rel=1e-15)  # / D_cur, not / D_prev (0.2)


def test_stop_rule_fires_on_a_converging_oracle_run():
    # the joint iteration on a tiny problem: the objective decreases
    # monotonically, and the rule fires where the decrease first drops to eps
    V, W, H = _small(seed=5, F=8, N=9, K=2)
    trace = [O.objective(V, W, H, 1.0)]
    for _ in range(400):
        W, H = O.jmm_iteration(V, W, H, 1.0)
        trace.append(O.objective(V, W, H, 1.0))
    t = O.stop_iteration(trace, 1e-5)
    assert t is not None
    rd = [(trace[i - 1] - trace[i]) / trace[i] for i in range(1, t + 1)]
    assert all(r > 1e-5 for r in rd[:-1]) and rd[-1] <= 1e-5
