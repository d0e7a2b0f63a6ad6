"""FP64 CPU oracle for beta-NMF by majorization-minimization (MM).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference
that the GPU library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path never
does.  It shares no code with the GPU library (no kernels, headers, helpers or
constant tables) and imports nothing from it.

Everything is float64 NumPy.  Inputs are taken as given (callers pass the
float32 data promoted to float64, so both sides see the same numbers).

Paper: "Joint Majorization-Minimization for Nonnegative Matrix Factorization
with the beta-divergence" (Marmin, Goulart, Fevotte).

Contents, each following the passage cited in its docstring:

* ``beta_divergence`` / ``objective``   -- Sec. 2.1, eqs. (obj_fct) and (beta-div)
* ``gamma_exponent``                    -- Sec. 2.2, eq. (def_gamma); ``exponent="one"`` in the
                                           two iterations replaces it by 1 (the heuristic of
                                           Sec. 3.3.3, "Failure of heuristic updates")
* ``chi1`` / ``chi2``                   -- Sec. 3.2, definitions under eq. (jnt_update)
* ``bmm_iteration``                     -- Sec. 2.2, eq. (alt_update) and Algorithm 1 (BMM)
* ``jmm_iteration``                     -- Sec. 3.2, eq. (jnt_update) and Algorithm 2 (JMM)
* ``normalize``                         -- Sec. 4.1.2 (scaling ambiguity removal)
* ``gradient``                          -- derivative of eq. (obj_fct); it is the quantity
                                           inside the KKT residuals of Sec. 4.1.5
* ``kkt_residuals``                     -- Sec. 4.1.5
* ``joint_auxiliary``                   -- Sec. 3.1, Table 1, eqs. (simplif) and (jointG)
* ``relative_decrease``                 -- Sec. 4.1.2 stopping criterion
* ``stop_iteration``                    -- Sec. 4.1.2: first outer iteration where it fires
* ``kl_sparse_objective`` /
  ``kl_sparse_iteration``               -- beta = 1 on a sparse V given by its nonzeros (CSR):
                                           the Table 2 (Sec. 3.3.1) KL updates of both methods,
                                           for count data such as the play counts of Sec. 4.4

Smoothing constant kappa (Sec. 4.1.3): the data V is replaced by V + kappa and
every product WH (or W~H~) by WH + kappa.  The paper gives no value; the
default here is 0.

Readings where the paper is silent (the same list is kept with the design notes):

* d_beta(0 | y) takes its limit: y for beta = 1, +inf for beta <= 0,
  y^beta / beta for beta > 0, beta != 1.
* x^0 is 1 (including 0^0) in every power that appears in the updates.
* A non-finite or zero-denominator ratio in an update is an error
  (``FloatingPointError``), never clamped.
* Normalization leaves a column of W whose norm is zero unchanged.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gamma_exponent",
    "beta_divergence",
    "objective",
    "chi1",
    "chi2",
    "bmm_iteration",
    "jmm_iteration",
    "normalize",
    "gradient",
    "kkt_residuals",
    "joint_auxiliary",
    "relative_decrease",
    "stop_iteration",
    "kl_sparse_objective",
    "kl_sparse_iteration",
]


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def _pow(x, p):
    """Entry-wise x**p with the convention x**0 == 1 (also for x == 0)."""
    x = _f64(x)
    if p == 0.0:
        return np.ones_like(x)
    with np.errstate(divide="ignore"):
        return np.power(x, p)


def gamma_exponent(beta: float) -> float:
    """Exponent gamma(beta) of the multiplicative updates, eq. (def_gamma), Sec. 2.2.

    1/(2-beta) below 1, 1 on [1, 2], 1/(beta-1) above 2.
    """
    beta = float(beta)
    if beta < 1.0:
        return 1.0 / (2.0 - beta)
    if beta <= 2.0:
        return 1.0
    return 1.0 / (beta - 1.0)


def beta_divergence(x, y, beta: float):
    """Entry-wise beta-divergence d_beta(x | y), eq. (beta-div), Sec. 2.1.

    beta = 1: x log(x/y) - x + y (Kullback-Leibler); beta = 0: x/y - log(x/y) - 1
    (Itakura-Saito); otherwise x^b/(b(b-1)) + y^b/b - x y^(b-1)/(b-1).
    At x = 0 the limit of the expression is taken (see the module notes).
    """
    x = _f64(x)
    y = _f64(y)
    x, y = np.broadcast_arrays(x, y)
    beta = float(beta)
    out = np.empty(x.shape, dtype=np.float64)
    pos = x > 0
    if beta == 1.0:
        xp, yp = x[pos], y[pos]
        out[pos] = xp * np.log(xp / yp) - xp + yp
        out[~pos] = y[~pos]
    elif beta == 0.0:
        xp, yp = x[pos], y[pos]
        out[pos] = xp / yp - np.log(xp / yp) - 1.0
        out[~pos] = np.inf
    else:
        b = beta
        xp, yp = x[pos], y[pos]
        out[pos] = xp ** b / (b * (b - 1.0)) + yp ** b / b - xp * yp ** (b - 1.0) / (b - 1.0)
        if b > 0:
            out[~pos] = y[~pos] ** b / b
        else:
            out[~pos] = np.inf
    return out


def objective(V, W, H, beta: float, kappa: float = 0.0) -> float:
    """D_beta(V + kappa | WH + kappa): the separable sum of eq. (obj_fct), Sec. 2.1 / 4.1.3."""
    V = _f64(V)
    L = _f64(W) @ _f64(H)
    return float(np.sum(beta_divergence(V + kappa, L + kappa, beta)))


def chi1(M, Mt, beta: float):
    """chi_{1,beta}(M, M~) of Sec. 3.2: M~^(2-beta) / M^(1-beta) for beta <= 2, else M."""
    M = _f64(M)
    Mt = _f64(Mt)
    if beta <= 2.0:
        return _pow(Mt, 2.0 - beta) / _pow(M, 1.0 - beta)
    return M.copy()


def chi2(M, Mt, beta: float):
    """chi_{2,beta}(M, M~) of Sec. 3.2: M for beta < 1, else M^beta / M~^(beta-1)."""
    M = _f64(M)
    Mt = _f64(Mt)
    if beta < 1.0:
        return M.copy()
    return _pow(M, beta) / _pow(Mt, beta - 1.0)


def _ratio(num, den, g):
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        r = num / den
    if not np.all(np.isfinite(r)) or np.any(den == 0):
        raise FloatingPointError("multiplicative update ratio is not finite")
    return _pow(r, g)


def normalize(W, H):
    """Divide each column of W by its l2 norm and scale the rows of H accordingly (Sec. 4.1.2).

    A zero column is left unchanged.  WH is unchanged by construction.
    """
    W = _f64(W).copy()
    H = _f64(H).copy()
    n = np.sqrt(np.sum(W * W, axis=0))
    nz = n > 0
    W[:, nz] /= n[nz]
    H[nz, :] *= n[nz, None]
    return W, H


def _exponent(beta: float, exponent: str) -> float:
    """gamma(beta) (``"mm"``), or 1 for every beta (``"one"``: the heuristic that
    sets gamma(beta) to 1 in the update even outside [1, 2], discussed for both
    methods in Sec. 3.3.3, "Failure of heuristic updates")."""
    if exponent == "mm":
        return gamma_exponent(beta)
    if exponent == "one":
        return 1.0
    raise ValueError(exponent)


def bmm_iteration(V, W, H, beta: float, L_W: int = 1, L_H: int = 1, kappa: float = 0.0,
                  norm: bool = True, return_parts: bool = False, exponent: str = "mm"):
    """One outer iteration of block MM (Algorithm 1, Sec. 2.2), eq. (alt_update).

    L_W multiplicative updates of W against the current H (each recomputes WH),
    then L_H updates of H against the new W.  Optional column normalization at
    the end (Sec. 4.1.2).  With ``return_parts`` the numerators/denominators of
    the last W and H sub-iteration are returned as well.  ``exponent``: see
    ``_exponent``.
    """
    V = _f64(V) + kappa
    W = _f64(W).copy()
    H = _f64(H).copy()
    g = _exponent(beta, exponent)
    for _ in range(L_W):
        Lam = W @ H + kappa
        numW = (_pow(Lam, beta - 2.0) * V) @ H.T
        denW = _pow(Lam, beta - 1.0) @ H.T
        W = W * _ratio(numW, denW, g)
    for _ in range(L_H):
        Lam = W @ H + kappa
        numH = W.T @ (_pow(Lam, beta - 2.0) * V)
        denH = W.T @ _pow(Lam, beta - 1.0)
        H = H * _ratio(numH, denH, g)
    Wn, Hn = (normalize(W, H) if norm else (W, H))
    if return_parts:
        return Wn, Hn, dict(numW=numW, denW=denW, numH=numH, denH=denH, W_unnorm=W, H_unnorm=H)
    return Wn, Hn


def jmm_iteration(V, Wt, Ht, beta: float, L: int = 1, kappa: float = 0.0, norm: bool = True,
                  return_parts: bool = False, exponent: str = "mm"):
    """One outer iteration of joint MM (Algorithm 2, Sec. 3.2), eq. (jnt_update).

    V~ = W~ H~ (+ kappa) is formed once.  The L sub-iterations update W and then
    H, always multiplying the *tilde* iterates, with chi_1/chi_2 evaluated at the
    latest sub-iterate and the tilde iterate.  Optional normalization at the end.
    ``exponent``: see ``_exponent``.
    """
    V = _f64(V) + kappa
    Wt = _f64(Wt)
    Ht = _f64(Ht)
    g = _exponent(beta, exponent)
    Vt = Wt @ Ht + kappa
    P = V / _pow(Vt, 2.0 - beta)          # V / V~^(2-beta)
    Q = _pow(Vt, beta - 1.0)              # V~^(beta-1)
    W, H = Wt.copy(), Ht.copy()
    for _ in range(L):
        numW = P @ chi1(H, Ht, beta).T
        denW = Q @ chi2(H, Ht, beta).T
        W = Wt * _ratio(numW, denW, g)
        numH = chi1(W, Wt, beta).T @ P
        denH = chi2(W, Wt, beta).T @ Q
        H = Ht * _ratio(numH, denH, g)
    Wn, Hn = (normalize(W, H) if norm else (W, H))
    if return_parts:
        return Wn, Hn, dict(numW=numW, denW=denW, numH=numH, denH=denH, W_unnorm=W, H_unnorm=H)
    return Wn, Hn


def gradient(V, W, H, beta: float, kappa: float = 0.0):
    """Gradient of D_beta(V + kappa | WH + kappa) w.r.t. W and H.

    With Lam = WH + kappa and E = Lam^(beta-2) * (Lam - V - kappa) (the derivative
    of d_beta in its second argument), grad_W = E H^T and grad_H = W^T E.  These
    are the bracketed terms of the KKT residuals in Sec. 4.1.5.
    """
    V = _f64(V)
    W = _f64(W)
    H = _f64(H)
    Lam = W @ H + kappa
    E = _pow(Lam, beta - 2.0) * (Lam - (V + kappa))
    return E @ H.T, W.T @ E


def kkt_residuals(V, W, H, beta: float, kappa: float = 0.0):
    """res(W), res(H) of Sec. 4.1.5.

    res(W) = || min(W, grad_W D) ||_1 / (F K) and res(H) = || min(H, grad_H D) ||_1 / (K N):
    the entry-wise minimum of each factor and its gradient (the bracketed
    (WH)^(beta-2) (WH - V) terms contracted with H^T, resp. W^T), its l1 norm
    (sum of absolute values), divided by the number of entries of that factor.
    """
    gW, gH = gradient(V, W, H, beta, kappa)
    W = _f64(W)
    H = _f64(H)
    rW = float(np.sum(np.abs(np.minimum(W, gW)))) / W.size
    rH = float(np.sum(np.abs(np.minimum(H, gH)))) / H.size
    return rW, rH


def _split_terms(v, y, beta):
    """Convex, concave and constant parts of d_beta(v | y) in y, Table 1 (Sec. 3.1).

    Returns three callables of y (for fixed v) plus the derivative of the concave part.
    """
    b = float(beta)
    if b == 0.0:
        conv = lambda t: v / t
        conc = lambda t: np.log(t)
        dconc = lambda t: 1.0 / t
        const = -(np.log(v) + 1.0)
    elif 1.0 <= b <= 2.0:
        conv = lambda t: beta_divergence(v, t, b)
        conc = lambda t: np.zeros_like(_f64(t))
        dconc = lambda t: np.zeros_like(_f64(t))
        const = np.zeros_like(_f64(v))
    elif b < 1.0:
        conv = lambda t: -v * _pow(t, b - 1.0) / (b - 1.0)
        conc = lambda t: _pow(t, b) / b
        dconc = lambda t: _pow(t, b - 1.0)
        const = _pow(v, b) / (b * (b - 1.0))
    else:
        conv = lambda t: _pow(t, b) / b
        conc = lambda t: -v * _pow(t, b - 1.0) / (b - 1.0)
        dconc = lambda t: -v * _pow(t, b - 2.0)
        const = _pow(v, b) / (b * (b - 1.0))
    return conv, conc, dconc, const


def joint_auxiliary(V, W, H, Wt, Ht, beta: float) -> float:
    """Joint auxiliary function G(W, H | W~, H~) of eq. (jointG), Sec. 3.1.

    Convex part majorized by Jensen's inequality with weights
    lam~_fnk = w~_fk h~_kn / v~_fn, v~ = [W~H~]_fn (eq. simplif); concave part by
    its tangent at v~_fn; constant part unchanged.  Materializes an F x N x K
    array: tiny inputs only.
    """
    V = _f64(V)
    W, H, Wt, Ht = (_f64(a) for a in (W, H, Wt, Ht))
    Vt = Wt @ Ht
    lam = Wt[:, None, :] * Ht.T[None, :, :] / Vt[:, :, None]          # F x N x K
    prod = W[:, None, :] * H.T[None, :, :]                             # w_fk h_kn
    conv, conc, dconc, const = _split_terms(V[:, :, None], None, beta)
    Gconv = np.sum(lam * conv(prod / lam), axis=2)
    conv2, conc2, dconc2, const2 = _split_terms(V, None, beta)
    Gconc = conc2(Vt) + dconc2(Vt) * (W @ H - Vt)
    return float(np.sum(Gconv + Gconc + const2))


def relative_decrease(D_prev: float, D_cur: float) -> float:
    """(D(previous iterate) - D(current iterate)) / D(current iterate), Sec. 4.1.2.

    Positive when the objective went down.  The paper prints no absolute value,
    so an increase gives a negative value, which is below any tolerance.
    """
    return (D_prev - D_cur) / D_cur


def stop_iteration(trace, eps: float = 1e-5):
    """Stopping rule of Sec. 4.1.2 applied to an objective trace.

    ``trace[t]`` is D_beta at the outer iterate t (t = 0 the initialization).
    Returns the first t >= 1 with relative_decrease(trace[t-1], trace[t]) <= eps:
    the algorithm stops there and iterate t is the one it returns.  None when
    the rule does not fire within the trace.  The paper's tolerance is 1e-5.
    """
    for t in range(1, len(trace)):
        if relative_decrease(float(trace[t - 1]), float(trace[t])) <= eps:
            return t
    return None


# ---------------------------------------------------------------------------
# beta = 1 (Kullback-Leibler) with V stored by its nonzeros
# ---------------------------------------------------------------------------
def _csr_rows(row_ptr, col_idx, vals):
    """(f, columns, values) of every row of a CSR matrix, in row order."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    for f in range(len(row_ptr) - 1):
        a, b = row_ptr[f], row_ptr[f + 1]
        yield f, np.asarray(col_idx[a:b], dtype=np.int64), _f64(vals[a:b])


def kl_sparse_objective(row_ptr, col_idx, vals, W, H) -> float:
    """D_1(V | WH) of eqs. (obj_fct), (beta-div) at beta = 1 for V given in CSR form.

    Every entry contributes [WH]_fn (the y term of d_1); an entry with v > 0
    adds v log(v / [WH]_fn) - v, and v = 0 adds nothing more (the limit
    0 log 0 = 0).  So only the stored nonzeros need [WH]_fn, and the sum of all
    [WH]_fn is sum_k (sum_f w_fk)(sum_n h_kn).
    """
    W = _f64(W)
    H = _f64(H)
    total = float(np.sum(W.sum(axis=0) * H.sum(axis=1)))
    for f, cols, v in _csr_rows(row_ptr, col_idx, vals):
        keep = v > 0
        cols, v = cols[keep], v[keep]
        lam = H[:, cols].T @ W[f]                      # [WH]_fn at the row's nonzeros
        total += float(np.sum(v * np.log(v / lam) - v))
    return total


def _kl_ratio_terms(row_ptr, col_idx, vals, Wl, Hl):
    """P = V / (Wl Hl) at the stored entries, in CSR order (0 where v = 0)."""
    out = []
    for f, cols, v in _csr_rows(row_ptr, col_idx, vals):
        lam = Hl[:, cols].T @ Wl[f]
        out.append(v / lam)
    return out


def kl_sparse_iteration(row_ptr, col_idx, vals, W, H, mode: str = "joint", norm: bool = True):
    """One outer iteration at beta = 1 (gamma = 1) for V given in CSR form.

    Table 2 (Sec. 3.3.1), KL row, with V / (WH) needed only where v != 0:

    * both methods, W step: numW = P H~^T with P = V / (W~ H~) at the nonzeros,
      denW = 1 H~^T, i.e. the row sums of H~ for every row of W;
    * joint MM (Algorithm 2, L = 1): chi_1(W, W~) = W~ and chi_2(W, W~) = W at
      beta = 1, so numH = W~^T P with the same P, denH = W_new^T 1, the column
      sums of W_new; H_new = H~ numH / denH;
    * alternating MU (Algorithm 1): numH = W_new^T P' with P' = V / (W_new H~),
      denH = the column sums of W_new.

    Optional normalization (Sec. 4.1.2) at the end.  An undefined ratio raises
    FloatingPointError, as in the dense iterations.
    """
    if mode not in ("joint", "alternating"):
        raise ValueError(mode)
    Wt = _f64(W)
    Ht = _f64(H)
    F, K = Wt.shape
    N = Ht.shape[1]
    P = _kl_ratio_terms(row_ptr, col_idx, vals, Wt, Ht)
    numW = np.zeros((F, K))
    for (f, cols, _), p in zip(_csr_rows(row_ptr, col_idx, vals), P):
        numW[f] = Ht[:, cols] @ p
    denW = np.broadcast_to(Ht.sum(axis=1), (F, K))
    Wn = Wt * _ratio(numW, denW, 1.0)
    if mode == "alternating":
        P = _kl_ratio_terms(row_ptr, col_idx, vals, Wn, Ht)
        chi = Wn
    else:
        chi = Wt
    numH = np.zeros((K, N))
    for (f, cols, _), p in zip(_csr_rows(row_ptr, col_idx, vals), P):
        numH[:, cols] += np.outer(chi[f], p)      # column scatter of chi_1[f, k] p_fn
    denH = np.broadcast_to(Wn.sum(axis=0)[:, None], (K, N))
    Hn = Ht * _ratio(numH, denH, 1.0)
    return normalize(Wn, Hn) if norm else (Wn, Hn)
