"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/nmf_beta.h, and rejects bad arguments with
the documented status codes before any device work."""
import ctypes
import os
import re

import pytest

import paper_2106_15214_amd as nb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmf_beta.h")

OK, E_NULL, E_SHAPE, E_BETA, E_ALIAS, E_WS, E_HIP, E_UNSUP, E_ARG, E_NODEV = range(10)


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nmf_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = nb.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = nb.lib()
    for st in range(10):
        s = L.nmf_status_string(st).decode()
        assert s.startswith("NMF_")
    assert L.nmf_status_string(99).decode() == "unknown nmf_status"
    assert b"gfx950" in L.nmf_version()


def test_step_argument_checks():
    c = nb.check_step_args
    assert c(100, 200, 10) == OK
    assert c(0, 200, 10) == E_SHAPE
    assert c(100, 0, 10) == E_SHAPE
    assert c(100, 200, 0) == E_SHAPE
    assert c(100, 200, 129) == E_UNSUP
    assert c(100, 200, 128) == OK
    assert c(100, 200, 10, ldv=199) == E_SHAPE
    assert c(100, 200, 10, ldw=9) == E_SHAPE
    assert c(100, 200, 10, ldh=150) == E_SHAPE
    assert c(100, 200, 10, V=0) == E_NULL
    assert c(100, 200, 10, W=0) == E_NULL
    assert c(100, 200, 10, beta=float("nan")) == E_BETA
    assert c(100, 200, 10, beta=float("inf")) == E_BETA
    assert c(100, 200, 10, mode=2) == E_ARG
    assert c(100, 200, 10, kappa=-1.0) == E_BETA
    assert c(100, 200, 10, inner_iters=2) == OK
    assert c(100, 200, 10, inner_iters=2, mode=0) == OK
    # joint sub-iterations keep P and Q: at most 2^28 entries of V
    far = dict(V=1 << 36, W=1 << 38, H=1 << 39)  # a 1.6 GB V must not overlap W, H
    assert c(20000, 20000, 10, inner_iters=2, **far) == E_UNSUP
    assert c(20000, 20000, 10, inner_iters=2, mode=0, **far) == OK
    assert c(100, 200, 10, inner_iters=2, precision=1) == E_UNSUP
    assert c(100, 200, 10, inner_iters=3, mode=0, precision=1) == OK
    assert c(100, 200, 10, inner_iters=0, mode=0) == E_ARG
    assert c(100, 200, 10, inner_iters=1001, mode=0) == E_ARG
    assert c(100, 200, 10, precision=7) == E_UNSUP
    assert c(100, 200, 10, exponent="one") == OK
    assert c(100, 200, 10, exponent=2) == E_ARG
    assert c(100, 200, 10, exponent=-1) == E_ARG


def test_alias_detection():
    c = nb.check_step_args
    V = 0x10000000
    # W placed inside V's span
    assert c(100, 200, 10, V=V, W=V + 4 * 200 * 50) == E_ALIAS
    # H right after V's last element: no overlap
    assert c(100, 200, 10, V=V, H=V + 4 * 200 * 100) == OK
    # one element earlier overlaps
    assert c(100, 200, 10, V=V, H=V + 4 * (200 * 100 - 1)) == E_ALIAS


def test_null_context_and_pointers():
    L = nb.lib()
    assert L.nmf_create(None, 0) == E_NULL
    assert L.nmf_destroy(None) == E_NULL
    assert L.nmf_reserve(None, 1, 1, 1) == E_NULL
    f = ctypes.c_uint32()
    assert L.nmf_get_flags(None, None, ctypes.byref(f), 0) == E_NULL
    assert L.nmf_beta_step(None, None, 1, 1, 1, 1, 1, 2, 1, 3, 1, 1.0, 1, None, None) == E_NULL


def test_create_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert nb.lib().nmf_create(ctypes.byref(h), 0) == E_NODEV
    assert not h.value
    with pytest.raises(nb.NmfError):
        nb.Context(0)


def test_binding_rejects_host_tensors():
    import torch
    V = torch.ones(4, 5)
    W = torch.ones(4, 2)
    H = torch.ones(2, 5)
    with pytest.raises((ValueError, nb.NmfError, RuntimeError)):
        nb.step(V, W, H, 1.0, "joint", ctx=object.__new__(nb.Context))
