"""Seeded synthetic inputs for beta-NMF workloads.

This module only draws random numbers and assembles matrices; it contains none
of the factorization method's arithmetic (no divergence, no update rule).  It is
the single source of inputs shared by the CPU oracle tests, the GPU parity
tests and the benchmark, so both sides of every comparison see identical data.

Every generator returns float32 C-contiguous arrays (the GPU's storage type);
the oracle promotes them to float64.  Large matrices are generated in
independent row blocks, each with its own child seed, so any row range (for
example a crop of the count-data matrix) can be regenerated without drawing the
whole matrix.

Workloads (shapes and distributions of the paper's experiments, with synthetic
data standing in for the real datasets, which are not available):

* ``tiny_kl``      F=64,    N=100,   K=5,  beta=1,   V = Poisson(W0 H0), W0,H0 ~ Gamma(1,1)
* ``faces_euc``    F=361,   N=2429,  K=49, beta=2,   V = clip(W0 H0 + N(0, 0.01^2), 0, inf) / max,
                   W0,H0 ~ Gamma(0.5,1)  (stands in for the face-image experiment)
* ``spectro_is``   F=513,   N=6000,  K=20, beta in {0, 0.5}, V = (W0 H0) * E, E ~ Exp(1),
                   W0,H0 ~ Gamma(1,1)  (stands in for the audio spectrogram experiment)
* ``counts_kl``    F=20000, N=10000, K=50, beta=1,   V = Poisson(0.02 W0 H0), W0,H0 ~ Gamma(0.3,1)
                   (stands in for the song play-count experiment; about 8.5 % nonzeros)
* ``counts_kl_sparse``  the same with V = Poisson(0.0022 W0 H0): about 1 % nonzeros, closer
                   to the play-count data's density; used in CSR form by the sparse path
* ``batched``      512 problems, F ~ U{128..1025}, N ~ U{200..5000}, K ~ U{8..64},
                   beta in {0, .5, 1, 1.5, 2}, Poisson or Gamma-noised V

Initial factors are Uniform(0.1, 1); for every workload except ``tiny_kl`` they
are then multiplied by one common scalar s = sqrt(mean(V) / mean(W H)) so the
first iterate has the data's scale.  mean(W H) is obtained from column/row sums
(mean(WH) = sum_k colsum(W)_k rowsum(H)_k / (F N)), not from the product.
"""
from __future__ import annotations

import dataclasses
from typing import Iterator, List, Optional, Tuple

import numpy as np

__all__ = [
    "Problem",
    "WORKLOADS",
    "make_problem",
    "make_factors",
    "make_init",
    "v_rows",
    "batched_specs",
    "make_batched_problem",
    "random_positive",
    "to_csr",
    "to_csc",
]

_ROW_BLOCK = 512  # rows per independently seeded block of V


@dataclasses.dataclass
class Problem:
    """One NMF instance: data V (F x N), init (W, H), divergence parameter beta."""

    name: str
    V: np.ndarray
    W: np.ndarray
    H: np.ndarray
    beta: float
    iters: int

    @property
    def shape(self) -> Tuple[int, int, int]:
        return self.V.shape[0], self.V.shape[1], self.W.shape[1]


# name -> (F, N, K, default beta, iterations, data seed)
WORKLOADS = {
    "tiny_kl": (64, 100, 5, 1.0, 100, 1),
    "faces_euc": (361, 2429, 49, 2.0, 500, 2),
    "spectro_is": (513, 6000, 20, 0.0, 300, 3),
    "counts_kl": (20000, 10000, 50, 1.0, 5, 4),
    "counts_kl_sparse": (20000, 10000, 50, 1.0, 5, 4),
}
# Poisson rate scale of the count workloads
_COUNT_SCALE = {"counts_kl": 0.02, "counts_kl_sparse": 0.0022}


def _seq(seed: int, *key: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([int(seed), *[int(k) for k in key]])


def make_factors(name: str, F: int, N: int, K: int, seed: int) -> Tuple[np.ndarray, np.ndarray]:
    """Ground-truth factors W0 (F x K) and H0 (K x N), float64."""
    shape = {"tiny_kl": 1.0, "faces_euc": 0.5, "spectro_is": 1.0, "counts_kl": 0.3, "counts_kl_sparse": 0.3}[name]
    rng = np.random.default_rng(_seq(seed, 0))
    W0 = rng.gamma(shape, 1.0, size=(F, K))
    H0 = rng.gamma(shape, 1.0, size=(K, N))
    return W0, H0


def _noise_block(name: str, L: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    if name == "tiny_kl":
        return rng.poisson(L).astype(np.float64)
    if name == "faces_euc":
        return np.clip(L + rng.normal(0.0, 0.01, size=L.shape), 0.0, np.inf)
    if name == "spectro_is":
        # Exp(1) on the open interval: a zero draw is replaced by the smallest positive double
        E = rng.exponential(1.0, size=L.shape)
        E[E == 0.0] = np.finfo(np.float64).tiny
        return L * E
    if name in _COUNT_SCALE:
        return rng.poisson(_COUNT_SCALE[name] * L).astype(np.float64)
    raise KeyError(name)


def v_rows(name: str, r0: int, r1: int, seed: Optional[int] = None) -> np.ndarray:
    """Rows r0:r1 of the workload's raw (unscaled) data matrix, float64.

    Rows are drawn in fixed blocks of ``_ROW_BLOCK`` with per-block seeds, so the
    result does not depend on which range is requested.
    """
    F, N, K, _, _, dseed = WORKLOADS[name]
    seed = dseed if seed is None else seed
    W0, H0 = make_factors(name, F, N, K, seed)
    out = np.empty((r1 - r0, N), dtype=np.float64)
    b0, b1 = r0 // _ROW_BLOCK, (r1 - 1) // _ROW_BLOCK
    for b in range(b0, b1 + 1):
        lo, hi = b * _ROW_BLOCK, min(F, (b + 1) * _ROW_BLOCK)
        rng = np.random.default_rng(_seq(seed, 1, b))
        blk = _noise_block(name, W0[lo:hi] @ H0, rng)
        s0, s1 = max(lo, r0), min(hi, r1)
        out[s0 - r0 : s1 - r0] = blk[s0 - lo : s1 - lo]
    return out


def make_init(F: int, N: int, K: int, seed: int, V: Optional[np.ndarray] = None,
              v_mean: Optional[float] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Uniform(0.1, 1) initial factors (float64), optionally rescaled to V's mean."""
    rng = np.random.default_rng(_seq(seed, 2))
    W = rng.uniform(0.1, 1.0, size=(F, K))
    H = rng.uniform(0.1, 1.0, size=(K, N))
    if v_mean is None and V is not None:
        v_mean = float(np.mean(V, dtype=np.float64))
    if v_mean is not None:
        wh_mean = float(W.sum(axis=0) @ H.sum(axis=1)) / (F * N)
        s = np.sqrt(v_mean / wh_mean)
        W *= s
        H *= s
    return W, H


def make_problem(name: str, seed: Optional[int] = None, init_seed: int = 1,
                 rows: Optional[Tuple[int, int]] = None,
                 cols: Optional[Tuple[int, int]] = None,
                 beta: Optional[float] = None) -> Problem:
    """Build a named workload (optionally a crop of it) as float32 arrays.

    ``rows``/``cols`` select a crop V[r0:r1, c0:c1] and the matching factor
    slices; the crop's data and init are the same numbers as in the full matrix.
    """
    F, N, K, b0, iters, dseed = WORKLOADS[name]
    seed = dseed if seed is None else seed
    r0, r1 = rows if rows is not None else (0, F)
    c0, c1 = cols if cols is not None else (0, N)
    V = v_rows(name, r0, r1, seed)[:, c0:c1]
    if name == "faces_euc":
        # rescale to [0, 1] by the maximum of the full matrix
        vmax = _faces_max(seed) if (rows is not None or cols is not None) else float(V.max())
        V = V / vmax
    Wf, Hf = make_init(F, N, K, init_seed)
    if name != "tiny_kl":
        vm = _full_mean(name, seed, V if rows is None and cols is None else None)
        wh_mean = float(Wf.sum(axis=0) @ Hf.sum(axis=1)) / (F * N)
        s = np.sqrt(vm / wh_mean)
        Wf *= s
        Hf *= s
    W = Wf[r0:r1]
    H = Hf[:, c0:c1]
    return Problem(name, np.ascontiguousarray(V, np.float32), np.ascontiguousarray(W, np.float32),
                   np.ascontiguousarray(H, np.float32), float(b0 if beta is None else beta), iters)


_MEAN_CACHE: dict = {}


def _full_mean(name: str, seed: int, V: Optional[np.ndarray]) -> float:
    key = (name, seed)
    if key not in _MEAN_CACHE:
        if name in _COUNT_SCALE:
            # expected mean of Poisson(c W0 H0): exact from the factors (no draw needed)
            F, N, K, *_ = WORKLOADS[name]
            W0, H0 = make_factors(name, F, N, K, seed)
            _MEAN_CACHE[key] = _COUNT_SCALE[name] * float(W0.sum(axis=0) @ H0.sum(axis=1)) / (F * N)
        elif V is not None:
            _MEAN_CACHE[key] = float(np.mean(V, dtype=np.float64))
        else:
            F = WORKLOADS[name][0]
            Vf = v_rows(name, 0, F, seed)
            if name == "faces_euc":
                Vf = Vf / Vf.max()
            _MEAN_CACHE[key] = float(np.mean(Vf))
    return _MEAN_CACHE[key]


def _faces_max(seed: int) -> float:
    key = ("faces_max", seed)
    if key not in _MEAN_CACHE:
        _MEAN_CACHE[key] = float(v_rows("faces_euc", 0, WORKLOADS["faces_euc"][0], seed).max())
    return _MEAN_CACHE[key]


# ---------------------------------------------------------------------------
# batched uneven problems
# ---------------------------------------------------------------------------
BATCH_BETAS = (0.0, 0.5, 1.0, 1.5, 2.0)


def batched_specs(count: int = 512, seed: int = 5) -> List[dict]:
    """Per-problem (F, N, K, beta, noise) draws for the batched workload."""
    rng = np.random.default_rng(_seq(seed, 7))
    specs = []
    for p in range(count):
        F = int(rng.integers(128, 1026))
        N = int(rng.integers(200, 5001))
        K = int(rng.integers(8, 65))
        beta = float(BATCH_BETAS[int(rng.integers(0, len(BATCH_BETAS)))])
        coin = int(rng.integers(0, 2))
        noise = "gamma" if (beta == 0.0 or coin == 1) else "poisson"
        specs.append(dict(F=F, N=N, K=K, beta=beta, noise=noise, seed=1000 + p))
    return specs


def make_batched_problem(spec: dict, scale: float = 1.0) -> Problem:
    """Data and init for one batched problem; ``scale`` shrinks F and N (for tests)."""
    F = max(1, int(round(spec["F"] * scale)))
    N = max(1, int(round(spec["N"] * scale)))
    K = spec["K"]
    rng = np.random.default_rng(_seq(spec["seed"], 3))
    W0 = rng.gamma(1.0, 1.0, size=(F, K))
    H0 = rng.gamma(1.0, 1.0, size=(K, N))
    L = W0 @ H0 / K
    if spec["noise"] == "poisson":
        V = rng.poisson(L).astype(np.float64)
    else:
        E = rng.exponential(1.0, size=L.shape)
        E[E == 0.0] = np.finfo(np.float64).tiny
        V = L * E
    W, H = make_init(F, N, K, spec["seed"], V=V)
    return Problem(f"batched{spec['seed']}", np.ascontiguousarray(V, np.float32),
                   np.ascontiguousarray(W, np.float32), np.ascontiguousarray(H, np.float32),
                   spec["beta"], 200)


def random_positive(F: int, N: int, K: int, seed: int, zeros: float = 0.0,
                    lo: float = 0.1, hi: float = 1.0) -> Problem:
    """Small generic instance for tests: V ~ Gamma(2, 0.5) with an optional zero fraction."""
    rng = np.random.default_rng(_seq(seed, 9))
    V = rng.gamma(2.0, 0.5, size=(F, N))
    if zeros > 0.0:
        V[rng.uniform(size=V.shape) < zeros] = 0.0
    W = rng.uniform(lo, hi, size=(F, K))
    H = rng.uniform(lo, hi, size=(K, N))
    return Problem(f"rand{seed}", np.ascontiguousarray(V, np.float32), np.ascontiguousarray(W, np.float32),
                   np.ascontiguousarray(H, np.float32), 1.0, 10)


def to_csr(V: np.ndarray):
    """Row-major compressed form of V's nonzero entries: (row_ptr int64[F + 1],
    col_idx int32[nnz], values float32[nnz]); columns ascend within a row."""
    V = np.asarray(V)
    rows, cols = np.nonzero(V)
    row_ptr = np.zeros(V.shape[0] + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=V.shape[0]), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), np.ascontiguousarray(V[rows, cols], dtype=np.float32)


def to_csc(V: np.ndarray):
    """Column-major compressed form of V's nonzero entries: (col_ptr int64[N + 1],
    row_idx int32[nnz], values float32[nnz]); rows ascend within a column."""
    return to_csr(np.asarray(V).T)
