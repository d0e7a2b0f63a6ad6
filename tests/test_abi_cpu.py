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

OK, E_NULL, E_SHAPE, E_BETA, E_ALIAS, E_WS, E_HIP, E_UNSUP, E_ARG, E_NODEV, E_IO = range(11)


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
    for st in range(11):
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


# ---------------------------------------------------------------------------
# batched step with device descriptors: host-only parts
# ---------------------------------------------------------------------------
# beta classes of the bucket rule as the header numbers them
_BETA_CLASS = {2.0: 1, 1.0: 2, 0.0: 3, 0.5: 4, 1.5: 5}


def _bucket_from_rule(F, N, K, beta):
    """The bucket rule as the header states it."""
    T = max(-(-F // 32), -(-N // 32))
    s = 0 if T <= 32 else 1 if T <= 64 else 2 if T <= 128 else 3
    k = 0 if K <= 32 else 1
    return 6 * (4 * k + s) + _BETA_CLASS.get(beta, 0)


def test_batch_bucket_rule():
    seen = set()
    for F, N, K in [(1, 1, 1), (1024, 1024, 32), (1025, 100, 32), (100, 2048, 33), (2049, 10, 64),
                    (4096, 4096, 64), (4097, 1, 1), (128, 5000, 17), (1000, 200, 64), (20000, 10000, 50),
                    (3000, 100, 10)]:
        for beta in (0.0, 0.5, 1.0, 1.5, 2.0, -0.5, 1.2, 2.5):
            b = nb.batch_bucket(F, N, K, beta)
            assert b == _bucket_from_rule(F, N, K, beta), (F, N, K, beta)
            seen.add(b)
    assert seen <= set(range(nb.BATCH_BUCKETS)) and len(seen) == nb.BATCH_BUCKETS
    for F, N, K, beta in [(0, 5, 5, 1.0), (5, 0, 5, 1.0), (5, 5, 0, 1.0), (5, 5, 65, 1.0), (5, 5, 5, float("nan")),
                          (5, 5, 5, float("inf"))]:
        assert nb.batch_bucket(F, N, K, beta) == -1


def _shapes(n, seed=3):
    import numpy as np
    rng = np.random.default_rng(seed)
    betas = (0.0, 0.5, 1.0, 1.5, 2.0)
    return [(int(rng.integers(128, 1026)), int(rng.integers(200, 5001)), int(rng.integers(8, 65)),
             betas[int(rng.integers(0, 5))]) for _ in range(n)]


def test_batch_requirements_invariants():
    shapes = _shapes(40)
    items, bytes_ = nb.batch_requirements(shapes, "joint")
    assert items > 0 and bytes_ > 0
    # additive over problems
    i1, b1 = nb.batch_requirements(shapes[:17], "joint")
    i2, b2 = nb.batch_requirements(shapes[17:], "joint")
    assert (i1 + i2, b1 + b2) == (items, bytes_)
    # the default table is 256 in every bucket
    assert nb.batch_requirements(shapes, "joint", [256] * 48) == (items, bytes_)
    # a table changed in one bucket changes the plans of that bucket's problems only
    b0 = _bucket_from_rule(*shapes[0])
    t = [256] * 48
    t[b0] = 4
    for sh in shapes:
        changed = nb.batch_requirements([sh], "joint", t) != nb.batch_requirements([sh], "joint")
        assert not changed or _bucket_from_rule(*sh) == b0, sh
    assert nb.batch_requirements(shapes[:1], "joint", t)[0] > nb.batch_requirements(shapes[:1], "joint")[0]
    # joint keeps P and Q per problem: more workspace, the same items
    ia, ba = nb.batch_requirements(shapes, "alternating")
    assert ia == items and ba < bytes_
    # fewer tiles per item: more items, never fewer bytes
    it, bt = nb.batch_requirements(shapes, "joint", [8] * 48)
    assert it > items and bt >= bytes_
    # a single problem: items are whole row / column blocks of 128 per pass
    (F, N, K) = (1000, 3000, 20)
    i, _ = nb.batch_requirements([(F, N, K, 1.0)], "joint", [4096] * 48)
    rb, cb = -(-F // 128), -(-N // 128)
    assert i >= rb + cb and i <= rb + cb + F + N
    # the item count phase by phase (row blocks of 128 x column groups, W-update
    # items of 64 rows, column blocks x row groups, H-update items of KP column
    # units of 256 / KP columns), written out from the splits: a problem whose
    # rows take one column group has no W-update items, and if its columns also
    # take one row group no H-update items either
    for (F2, N2, K2, t) in [(1000, 3000, 20, 256), (1000, 3000, 20, 128), (5000, 3000, 20, 128),
                            (1000, 3000, 20, 4), (700, 4500, 50, 100), (33, 1000, 8, 12)]:
        assert nb.batch_requirements([(F2, N2, K2, 0.5)], "joint", [t] * 48)[0] == _items_from_splits(F2, N2, K2, t)
        assert (nb.batch_requirements([(F2, N2, K2, 0.5)], "alternating", [t] * 48, precision="bf16")[0]
                == _items_from_splits(F2, N2, K2, t))


def test_batch_joint_keeps_pq_only_where_it_pays():
    """Workspace of one batched problem: joint MM keeps P, Q (an F x N tile
    store each) only at K > 32 and beta != 1, in either precision; elsewhere
    its H pass forms Lambda~ again and its workspace equals alternating MU's."""
    F, N = 700, 900
    pq = 2 * (-(-F // 32)) * (-(-N // 32)) * 32 * 32 * 4  # P and Q tiles, float32

    def ws(K, beta, mode, precision="fp32"):
        return nb.batch_requirements([(F, N, K, beta)], mode, precision=precision)[1]

    for K, beta in [(20, 0.5), (32, 2.0), (50, 1.0), (64, 1.0)]:
        assert ws(K, beta, "joint") == ws(K, beta, "alternating"), (K, beta)
    for K, beta in [(33, 0.5), (50, 0.0), (64, 2.0), (50, 1.5)]:
        assert ws(K, beta, "joint") - ws(K, beta, "alternating") >= pq, (K, beta)
    for K, beta in [(33, 0.5), (64, 2.0), (50, 0.0)]:
        assert ws(K, beta, "joint", "bf16") > ws(K, beta, "alternating", "bf16"), (K, beta)
    for K, beta in [(20, 0.5), (32, 1.0), (8, 2.0), (50, 1.0)]:
        assert ws(K, beta, "joint", "bf16") == ws(K, beta, "alternating", "bf16"), (K, beta)


def _groups(tiles_total, tiles):
    g = -(-tiles_total // tiles)
    per = -(-tiles_total // g)
    return -(-tiles_total // per)


def _items_from_splits(F, N, K, tiles):
    KP = 32 if K <= 32 else 64
    ng, fg = _groups(-(-N // 32), tiles), _groups(-(-F // 32), tiles)
    w_pass, h_pass = -(-F // 128) * ng, -(-N // 128) * fg
    w_update = 0 if ng == 1 else -(-F // 64)
    h_update = 0 if ng == 1 and fg == 1 else -(-(-(-N // (256 // KP))) // KP)
    return w_pass + w_update + h_pass + h_update


def test_batch_requirements_checks():
    with pytest.raises(nb.NmfError) as e:
        nb.batch_requirements([(10, 10, 65, 1.0)])
    assert e.value.status == E_UNSUP
    with pytest.raises(nb.NmfError) as e:
        nb.batch_requirements([(0, 10, 5, 1.0)])
    assert e.value.status == E_SHAPE
    with pytest.raises(nb.NmfError) as e:
        nb.batch_requirements([(10, 10, 5, 1.0)], "joint", [0] * 48)
    assert e.value.status == E_ARG
    with pytest.raises(nb.NmfError) as e:
        nb.batch_requirements([(10, 10, 5, float("nan"))])
    assert e.value.status == E_BETA
    L = nb.lib()
    n, b = ctypes.c_int64(), ctypes.c_int64()
    assert L.nmf_batch_requirements(None, 1, 1, 0, None, ctypes.byref(n), ctypes.byref(b)) == E_NULL
    arr = (nb._Problem * 1)(nb._Problem(10, 10, 5, None, 0, None, 0, None, 0, 1.0))
    assert L.nmf_batch_requirements(arr, 0, 1, 0, None, ctypes.byref(n), ctypes.byref(b)) == E_ARG
    assert L.nmf_batch_requirements(arr, 1, 5, 0, None, ctypes.byref(n), ctypes.byref(b)) == E_ARG
    assert L.nmf_batch_requirements(arr, 1, 1, 7, None, ctypes.byref(n), ctypes.byref(b)) == E_ARG
    assert L.nmf_batch_requirements(arr, 1, 1, 2, None, ctypes.byref(n), ctypes.byref(b)) == E_UNSUP  # FP16


def test_batched_entry_points_null_context():
    L = nb.lib()
    t = (ctypes.c_int32 * nb.BATCH_BUCKETS)()
    assert L.nmf_reserve_batched(None, 1, 1, 1) == E_NULL
    assert L.nmf_beta_step_batched(None, None, 1, 1, 1, None, None, None) == E_NULL
    assert L.nmf_set_batch_tiles(None, t) == E_NULL
    assert L.nmf_get_batch_tiles(None, t) == E_NULL
    arr = (nb._Problem * 1)()
    assert L.nmf_tune(None, None, arr, 1, 1, None, 1, None, t, None, None) == E_NULL
