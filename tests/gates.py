"""Parity gates shared by the GPU tests (HIP library vs the FP64 oracle).

Two measures of a computed factor X against the oracle's X_ref:

* ``rel``  -- Frobenius:    ||X - X_ref||_F / ||X_ref||_F
* ``elem`` -- entry-wise:   max |X - X_ref| / (|X_ref| + 1e-6 max|X_ref|)

Bars per product type (the derivation is in the design notes):

* float32 products:      Frobenius 1e-5, entry-wise 1e-4
* bfloat16 products:     Frobenius 3e-3, entry-wise 4 u (2 + |beta - 2|), u = 2^-9
* float16 products:      the same with u = 2^-11
"""
import numpy as np

FRO = {"fp32": 1e-5, "bf16": 3e-3, "fp16": 3e-3}
ELEM_FP32 = 1e-4
UNIT = {"bf16": 2.0 ** -9, "fp16": 2.0 ** -11}


def rel(a, b):
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def elem(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if b.size == 0:
        return 0.0
    floor = 1e-6 * float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b) / (np.abs(b) + floor)))


def elem_bar(precision="fp32", beta=1.0):
    if precision == "fp32":
        return ELEM_FP32
    return 4.0 * UNIT[precision] * (2.0 + abs(float(beta) - 2.0))


def check_factor(got, ref, precision="fp32", beta=1.0, what="X", fro=None, el=None):
    """Asserts both gates; returns (Frobenius, entry-wise) errors."""
    e_f, e_e = rel(got, ref), elem(got, ref)
    bf = FRO[precision] if fro is None else fro
    be = elem_bar(precision, beta) if el is None else el
    assert e_f <= bf, f"{what}: Frobenius rel err {e_f:.3e} > {bf:.1e}"
    assert e_e <= be, f"{what}: entry-wise rel err {e_e:.3e} > {be:.1e}"
    return e_f, e_e


def check_pair(W, H, Wr, Hr, precision="fp32", beta=1.0, tag="", fro=None, el=None):
    eW = check_factor(W, Wr, precision, beta, f"W {tag}", fro, el)
    eH = check_factor(H, Hr, precision, beta, f"H {tag}", fro, el)
    print(f"[gate] {tag} W fro {eW[0]:.2e} elem {eW[1]:.2e} | H fro {eH[0]:.2e} elem {eH[1]:.2e}", flush=True)
    return eW, eH
