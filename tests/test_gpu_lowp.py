"""GPU parity of the bfloat16 / float16 matrix-core mode against the FP64 oracle.

In this mode the W- and H-step contractions take single bfloat16 (float16)
operands with float32 accumulation, Lambda = WH is formed from split operands
(hi*hi + lo*hi + hi*lo, about 2^-16 relative), and the element-wise terms stay
in float32.  Gates:
  W, H: relative Frobenius error <= 3e-3 per step (both operands of each
        product rounded once: <= 2 * 2^-9 per term, and the update exponent
        gamma <= 1 does not amplify it), and entry-wise error
        <= 4 u (2 + |beta - 2|) with u = 2^-9 (bfloat16) or 2^-11 (float16):
        numerator and denominator each within 2u, the ratio within 4u, and the
        alternating H step sees W_new's error through Lambda' = W_new H~,
        raised to |beta - 2| by the element-wise power (tests/gates.py);
  objective: |D_gpu - D| <= max(1e-6 D, 2^-14 * S) with
        S = sum_fn |d/dLambda d_beta(v|Lambda)| * Lambda, the first-order change
        of D under a relative perturbation 2^-14 of every Lambda entry (four
        times the split error bound);
  trajectories: every objective decrease holds up to twice that evaluation
        bound plus a 1e-6 relative slack for the rounded step (the MM
        guarantee holds for the exact step only).
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
TOL_FACTOR = 3e-3
PRECS = ["bf16", "fp16"]
_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = nb.Context(0)
    return _CTX["c"]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def obj_bound(V, W, H, beta, kappa=0.0):
    """First-order objective change under a 2^-14 relative change of Lambda."""
    L = W.astype(np.float64) @ H.astype(np.float64) + kappa
    V = V.astype(np.float64)
    S = float(np.sum(np.abs(L ** (beta - 1.0) * (L - V))))
    return 2.0 ** -14 * S


FLAG_RANGE = 8
FP16_MAX = 65504.0


def fp16_peak(V, W, H, beta, kappa=0.0):
    """Largest element-wise term or factor entry the float16 products see."""
    L = W.astype(np.float64) @ H.astype(np.float64) + kappa
    Vk = V.astype(np.float64) + kappa
    return max(np.max(Vk * L ** (beta - 2.0)), np.max(L ** (beta - 1.0)), np.max(W), np.max(H))


def gpu_step(V, W, H, beta, mode, prec, kappa=0.0):
    Vd, Wd, Hd = dev(V), dev(W), dev(H)
    o = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    nb.step(Vd, Wd, Hd, beta, mode, precision=prec, kappa=kappa, objective_out=o, ctx=ctx())
    torch.cuda.synchronize()
    fl = nb.get_flags(clear=True, ctx=ctx())
    return Wd.cpu().numpy(), Hd.cpu().numpy(), o.item(), fl


def check(V, W, H, beta, mode, prec, kappa=0.0, tag=""):
    print(f"[lowp] {tag} F={V.shape[0]} N={V.shape[1]} K={W.shape[1]} beta={beta} mode={mode} prec={prec}",
          flush=True)
    Wg, Hg, dg, fl = gpu_step(V, W, H, beta, mode, prec, kappa)
    if prec == "fp16":
        # documented behaviour: operands beyond the float16 range raise the
        # range flag (the step's result is then not used).  The oracle's peak
        # predicts it up to the float32 rounding of the terms and the chi
        # factors, hence the band between half and the full range.
        peak = fp16_peak(V, W, H, beta, kappa)
        if peak > FP16_MAX:
            assert fl & FLAG_RANGE, f"peak {peak:.3e} but no range flag"
        if fl & FLAG_RANGE:
            assert peak > 0.5 * FP16_MAX, f"range flag with peak {peak:.3e}"
            print(f"[lowp]   float16 range exceeded (peak {peak:.3e}), flag raised; "
                  "the same inputs with bfloat16 products are checked instead", flush=True)
            return check(V, W, H, beta, mode, "bf16", kappa, tag + " (bf16 after fp16 range flag)")
    assert fl == 0, fl
    f = O.jmm_iteration if mode == "joint" else O.bmm_iteration
    Wr, Hr = f(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta, kappa=kappa)
    d0 = O.objective(V.astype(np.float64), W.astype(np.float64), H.astype(np.float64), beta, kappa)
    (eW, _), (eH, _) = check_pair(Wg, Hg, Wr, Hr, prec, beta, tag=tag)
    tol = max(1e-6 * abs(d0), obj_bound(V, W, H, beta, kappa))
    assert abs(dg - d0) <= tol, f"objective err {abs(dg - d0):.3e} > {tol:.3e}"
    return eW, eH


SHAPES = [(64, 100, 5), (200, 150, 20), (257, 300, 49), (130, 70, 64), (33, 1000, 8), (1, 40, 3), (40, 1, 3),
          (129, 129, 1), (96, 160, 32)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("beta", [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, -0.5])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("prec", PRECS)
def test_lowp_step_parity_shapes(shape, beta, mode, prec):
    F, N, K = shape
    p = synth.random_positive(F, N, K, seed=F * 7 + N + K, zeros=0.1 if beta > 0 else 0.0)
    check(p.V, p.W, p.H, beta, mode, prec, tag="shape")


@pytest.mark.parametrize("name,beta,crop", [
    ("spectro_is", 0.0, None),
    ("spectro_is", 0.5, None),
    ("faces_euc", 2.0, None),
    ("tiny_kl", 1.0, None),
    ("counts_kl", 1.0, ((0, 300), (0, 400))),
])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("prec", PRECS)
def test_lowp_workload_parity(name, beta, crop, mode, prec):
    p = synth.make_problem(name, beta=beta, rows=crop[0] if crop else None, cols=crop[1] if crop else None)
    check(p.V, p.W, p.H, beta, mode, prec, tag=name)


def test_lowp_rejects_k_above_64():
    p = synth.random_positive(50, 60, 65, seed=1)
    with pytest.raises(nb.NmfError):
        gpu_step(p.V, p.W, p.H, 1.0, "joint", "bf16")
    with pytest.raises(nb.NmfError):
        gpu_step(p.V, p.W, p.H, 1.0, "joint", "fp16")


def test_lowp_kappa():
    p = synth.random_positive(120, 90, 16, seed=2, zeros=0.2)
    check(p.V, p.W, p.H, 0.0, "joint", "bf16", kappa=1e-3, tag="kappa")


@pytest.mark.parametrize("beta", [0.0, 0.5])
@pytest.mark.parametrize("mode", ["joint", "alternating"])
@pytest.mark.parametrize("prec", PRECS)
def test_lowp_spectrogram_trajectory_monotone(beta, mode, prec):
    # 120 iterations of the 513 x 6000, K = 20 spectrogram-shaped problem; the
    # objective decreases at every step up to its evaluation error, and at
    # t = 60 one step is checked against the oracle.
    p = synth.make_problem("spectro_is", beta=beta)
    V, W, H = dev(p.V), dev(p.W), dev(p.H)
    trace, bounds = [], []
    for t in range(120):
        if t == 60:
            check(p.V, W.cpu().numpy(), H.cpu().numpy(), beta, mode, prec, tag=f"t={t}")
        if t % 20 == 0:
            bounds.append(obj_bound(p.V, W.cpu().numpy(), H.cpu().numpy(), beta))
        o = torch.zeros(1, dtype=torch.float64, device=DEV)
        nb.step(V, W, H, beta, mode, precision=prec, objective_out=o, ctx=ctx())
        trace.append(o.item())
    assert nb.get_flags(clear=True, ctx=ctx()) == 0
    trace = np.array(trace)
    eps = 2 * max(bounds) + 1e-6 * trace[:-1]
    inc = trace[1:] - trace[:-1]
    print(f"[lowp] trajectory decrease {trace[0]:.6e} -> {trace[-1]:.6e}, max increase {inc.max():.3e}", flush=True)
    assert np.all(inc <= eps), float(np.max(inc - eps))
    assert trace[-1] < 0.9 * trace[0]


@pytest.mark.parametrize("prec", PRECS)
def test_lowp_close_to_fp32_trajectory(prec):
    # 50 iterations from one start: the low-precision factors stay within a few
    # 1e-3 of the float32 run and its objective within 1e-3.
    p = synth.make_problem("spectro_is", beta=0.5)
    V = dev(p.V)
    runs = {}
    for pr in ("fp32", prec):
        W, H = dev(p.W), dev(p.H)
        o = torch.zeros(1, dtype=torch.float64, device=DEV)
        for _ in range(50):
            nb.step(V, W, H, 0.5, "joint", precision=pr, objective_out=o, ctx=ctx())
        runs[pr] = (W.cpu().numpy(), H.cpu().numpy(), o.item())
    a, b = runs["fp32"], runs[prec]
    assert abs(a[2] - b[2]) <= 1e-3 * a[2]
    assert rel(b[0] @ b[1], a[0].astype(np.float64) @ a[1]) <= 1e-2


def test_lowp_deterministic():
    p = synth.random_positive(300, 500, 40, seed=4)
    a = gpu_step(p.V, p.W, p.H, 1.5, "joint", "bf16")
    b = gpu_step(p.V, p.W, p.H, 1.5, "joint", "bf16")
    assert a[3] == 0 and b[3] == 0
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
