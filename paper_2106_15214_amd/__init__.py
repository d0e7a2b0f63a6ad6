"""Python binding of the MI355X beta-NMF library (``libnmfbeta.so``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Torch tensors supply device memory and the current HIP stream.
The library must be built (``python -m paper_2106_15214_amd.build`` or
``__graft_entry__.build()``); if it is missing, loading raises.

Calls mirror include/nmf_beta.h:

* :func:`step`       -- one outer iteration (alternating or joint MM), in place
* :func:`objective`  -- D_beta(V + kappa | WH + kappa) as a device float64 scalar
* :func:`grad`       -- gradient of D_beta w.r.t. W and H
* :func:`validate`   -- domain scan setting the sticky DOMAIN flag
* :func:`get_flags`  -- read (and clear) the sticky numeric flags
* :class:`BetaDivergence` -- ``torch.autograd.Function`` with the GPU backward
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Tuple

__all__ = [
    "NmfError", "lib", "library_path", "Context", "default_context",
    "ALTERNATING", "JOINT", "FP32", "BF16", "FP16", "EXPONENTS",
    "FLAG_NONFINITE", "FLAG_DOMAIN", "FLAG_BARRIER", "FLAG_RANGE", "KERNELS",
    "step", "step_noalloc", "run", "kkt", "objective", "grad", "SparseV", "kl_step_sparse", "kl_objective_sparse",
    "sparse_validate", "validate", "get_flags", "check_step_args", "Batch", "BATCH_BUCKETS", "batch_bucket",
    "set_batch_tiles", "get_batch_tiles", "tune", "batch_requirements", "reserve_batched", "DeviceProblems",
    "step_batched", "FLAG_SKIPPED",
    "BetaDivergence", "beta_divergence",
]

ALTERNATING, JOINT = 0, 1
FP32, BF16, FP16 = 0, 1, 2
FLAG_NONFINITE, FLAG_DOMAIN = 1, 2
KERNELS = {"sweep_w": 0, "update_w": 1, "sweep_h": 2, "update_h": 3, "fused_step": 5, "sparse_pass": 6,
           "sparse_cols": 7}
PATHS = {"auto": 0, "stream": 1, "fused": 2}
FLAG_BARRIER = 4
FLAG_RANGE = 8  # float16 mode: an operand outside the float16 range
FLAG_SKIPPED = 16  # step_batched updated nothing (invalid descriptor, overlap, over capacity)
BATCH_BUCKETS = 48
MODES = {"alternating": ALTERNATING, "bmm": ALTERNATING, "joint": JOINT, "jmm": JOINT}
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp16": FP16}
# update exponent: gamma(beta) (the MM step) or 1 (the heuristic of Sec. 3.3.3)
EXPONENTS = {"mm": 0, "one": 1}

_HERE = os.path.dirname(os.path.abspath(__file__))
# NMF_BETA_LIBRARY selects another build of the same library (the host-side
# sanitizer build of the CPU tests); by default the in-tree libnmfbeta.so
library_path = os.environ.get("NMF_BETA_LIBRARY") or os.path.join(_HERE, "libnmfbeta.so")


class NmfError(RuntimeError):
    """A non-OK status returned by the library."""

    def __init__(self, status: int, where: str = ""):
        self.status = int(status)
        msg = _status_string(self.status)
        super().__init__(f"{where}: {msg}" if where else msg)


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("kappa", ctypes.c_float),
                ("inner_iters", ctypes.c_int32), ("normalize", ctypes.c_int32),
                ("exponent", ctypes.c_int32), ("gram", ctypes.c_int32)]


class _Problem(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("V", ctypes.c_void_p), ("ldv", ctypes.c_int64),
                ("W", ctypes.c_void_p), ("ldw", ctypes.c_int64),
                ("H", ctypes.c_void_p), ("ldh", ctypes.c_int64),
                ("beta", ctypes.c_double)]


class _SparseV(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int64), ("N", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("row_val", ctypes.c_void_p),
                ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p), ("col_val", ctypes.c_void_p)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("tiles_per_item", ctypes.c_int32), ("workers", ctypes.c_int32), ("lag", ctypes.c_int32)]


_lib = None
_lock = threading.Lock()
_i64, _i32, _u32, _dbl, _flt, _vp = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                     ctypes.c_double, ctypes.c_float, ctypes.c_void_p)


def lib() -> ctypes.CDLL:
    """Loads libnmfbeta.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(library_path):
            raise RuntimeError(f"HIP library not built: {library_path} is missing "
                               "(run python -m paper_2106_15214_amd.build)")
        L = ctypes.CDLL(library_path)
        L.nmf_status_string.restype = ctypes.c_char_p
        L.nmf_status_string.argtypes = [ctypes.c_int]
        L.nmf_version.restype = ctypes.c_char_p
        L.nmf_default_opts.argtypes = [ctypes.POINTER(_Opts)]
        L.nmf_default_opts.restype = None
        L.nmf_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int]
        L.nmf_destroy.argtypes = [_vp]
        L.nmf_reserve.argtypes = [_vp, _i64, _i64, _i64]
        L.nmf_check_step_args.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                          _dbl, _i32, ctypes.POINTER(_Opts)]
        L.nmf_beta_step.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                    _dbl, _i32, ctypes.POINTER(_Opts), _vp]
        L.nmf_beta_step_noalloc.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                            _dbl, _i32, ctypes.POINTER(_Opts), _vp, _vp]
        L.nmf_beta_objective.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                         _dbl, _flt, _vp]
        L.nmf_beta_grad.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                    _dbl, _flt, _dbl, _vp, _vp, _i64, _vp, _i64, _vp]
        L.nmf_beta_kkt.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _dbl, _flt, _vp]
        L.nmf_beta_run.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _dbl, _i32,
                                   ctypes.POINTER(_Opts), _i32, _dbl, _vp, _vp]
        L.nmf_beta_validate.argtypes = [_vp, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64,
                                        _dbl, _flt]
        L.nmf_get_flags.argtypes = [_vp, _vp, ctypes.POINTER(_u32), _i32]
        L.nmf_profile_enable.argtypes = [_vp, _u32]
        L.nmf_profile_read.argtypes = [_vp, _i32, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]
        L.nmf_set_launch.argtypes = [_vp, _i32, _i32]
        L.nmf_set_path.argtypes = [_vp, _i32]
        L.nmf_profile_phases.argtypes = [_vp, _vp, ctypes.POINTER(_dbl), _i32]
        PS = ctypes.POINTER(_SparseV)
        L.nmf_kl_step_sparse.argtypes = [_vp, _vp, PS, _i64, _vp, _i64, _vp, _i64, _i32, ctypes.POINTER(_Opts), _vp]
        L.nmf_kl_objective_sparse.argtypes = [_vp, _vp, PS, _i64, _vp, _i64, _vp, _i64, _vp]
        L.nmf_sparse_validate.argtypes = [_vp, _vp, PS]
        PP, PC = ctypes.POINTER(_Problem), ctypes.POINTER(_BatchConfig)
        L.nmf_batch_create.argtypes = [_vp, PP, _i32, _i32, ctypes.POINTER(_Opts), PC, ctypes.POINTER(_vp)]
        L.nmf_batch_step.argtypes = [_vp, _vp, _vp]
        L.nmf_batch_get_flags.argtypes = [_vp, _vp, ctypes.POINTER(_u32), _i32]
        L.nmf_batch_info.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i64)]
        L.nmf_batch_destroy.argtypes = [_vp]
        PI = ctypes.POINTER(_i32)
        L.nmf_batch_bucket.argtypes = [_i64, _i64, _i64, _dbl]
        L.nmf_batch_bucket.restype = _i32
        L.nmf_set_batch_tiles.argtypes = [_vp, PI]
        L.nmf_get_batch_tiles.argtypes = [_vp, PI]
        L.nmf_tune.argtypes = [_vp, _vp, PP, _i32, _i32, ctypes.POINTER(_Opts), _i32, ctypes.c_char_p, PI,
                               ctypes.POINTER(_dbl), PI]
        L.nmf_batch_requirements.argtypes = [PP, _i32, _i32, _i32, PI, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]
        L.nmf_reserve_batched.argtypes = [_vp, _i32, _i64, _i64]
        L.nmf_beta_step_batched.argtypes = [_vp, _vp, _i32, _vp, _i32, ctypes.POINTER(_Opts), _vp, _vp]
        for name in ("nmf_create", "nmf_destroy", "nmf_reserve", "nmf_check_step_args", "nmf_beta_step",
                     "nmf_beta_step_noalloc", "nmf_beta_kkt", "nmf_beta_run",
                     "nmf_beta_objective", "nmf_beta_grad", "nmf_beta_validate", "nmf_get_flags",
                     "nmf_profile_enable", "nmf_profile_read", "nmf_set_launch", "nmf_set_path",
                     "nmf_profile_phases", "nmf_batch_create", "nmf_batch_step", "nmf_batch_get_flags",
                     "nmf_batch_info", "nmf_batch_destroy", "nmf_set_batch_tiles", "nmf_get_batch_tiles",
                     "nmf_tune", "nmf_batch_requirements", "nmf_reserve_batched", "nmf_beta_step_batched",
                     "nmf_kl_step_sparse",
                     "nmf_kl_objective_sparse", "nmf_sparse_validate"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _status_string(st: int) -> str:
    try:
        return lib().nmf_status_string(int(st)).decode()
    except Exception:  # pragma: no cover - library absent
        return f"status {st}"


def _check(st: int, where: str):
    if st != 0:
        raise NmfError(st, where)


def _opts(precision=FP32, kappa=0.0, inner_iters=1, normalize=True, exponent="mm", gram=False) -> _Opts:
    o = _Opts()
    lib().nmf_default_opts(ctypes.byref(o))
    o.precision = PRECISIONS.get(precision, precision) if isinstance(precision, str) else int(precision)
    o.kappa = float(kappa)
    o.inner_iters = int(inner_iters)
    o.normalize = 1 if normalize else 0
    o.exponent = EXPONENTS.get(exponent, exponent) if isinstance(exponent, str) else int(exponent)
    o.gram = 1 if gram else 0
    return o


class Context:
    """A library context (workspace owner) on one HIP device."""

    def __init__(self, device: int = 0):
        h = _vp()
        _check(lib().nmf_create(ctypes.byref(h), int(device)), "nmf_create")
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            lib().nmf_destroy(self.handle)
            self.handle = _vp()

    def reserve(self, F: int, N: int, K: int):
        _check(lib().nmf_reserve(self.handle, F, N, K), "nmf_reserve")

    def set_launch(self, target_blocks: int = 0, min_tiles: int = 0):
        _check(lib().nmf_set_launch(self.handle, target_blocks, min_tiles), "nmf_set_launch")

    def set_path(self, path="auto"):
        """Execution path of step(): "auto", "stream" (four launches) or "fused" (one)."""
        _check(lib().nmf_set_path(self.handle, PATHS[path] if isinstance(path, str) else int(path)), "nmf_set_path")

    def profile(self, kernels) -> None:
        mask = 0
        for k in kernels:
            mask |= 1 << (KERNELS[k] if isinstance(k, str) else int(k))
        _check(lib().nmf_profile_enable(self.handle, mask), "nmf_profile_enable")

    def profile_phases(self, stream=None):
        """Phase durations (us) of the last single-launch step: W pass, barrier,
        W update, barrier, H pass, barrier, H update."""
        arr = (_dbl * 7)()
        _check(lib().nmf_profile_phases(self.handle, _stream(stream), arr, 7), "nmf_profile_phases")
        return list(arr)

    def profile_read(self, kernel) -> Tuple[float, int]:
        ms, n = _dbl(), _i64()
        kid = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        _check(lib().nmf_profile_read(self.handle, kid, ctypes.byref(ms), ctypes.byref(n)), "nmf_profile_read")
        return ms.value, n.value

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


_contexts = {}


def default_context(device: Optional[int] = None) -> Context:
    import torch
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _contexts:
        _contexts[d] = Context(d)
    return _contexts[d]


def _mat(t, name, writable=False):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dim() != 2 or (t.stride(1) != 1 and t.shape[1] > 1):
        raise ValueError(f"{name} must be 2-D with unit column stride")
    if t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        # overlapping rows (expand, as_strided): no valid leading dimension
        raise ValueError(f"{name} has overlapping rows (row stride {t.stride(0)} < {t.shape[1]} columns)")
    return t.data_ptr(), (t.stride(0) if t.shape[0] > 1 else t.shape[1])


def _dev_f64(t, name, n=1):
    """Device pointer of a float64 cuda tensor with at least n contiguous entries."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or t.numel() < n:
        raise ValueError(f"{name} must be a float64 device tensor with at least {n} entries")
    if n > 1 and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        return _vp(torch.cuda.current_stream().cuda_stream)
    return _vp(getattr(stream, "cuda_stream", stream))


def _ctx(ctx):
    return (ctx or default_context()).handle


def check_step_args(F, N, K, V=0x10000000, ldv=None, W=0x50000000, ldw=None, H=0x90000000, ldh=None,
                    beta=1.0, mode=JOINT, **kw) -> int:
    """Host-only argument check (no GPU needed); returns the library's status code."""
    o = _opts(**kw)
    return lib().nmf_check_step_args(F, N, K, V, N if ldv is None else ldv, W, K if ldw is None else ldw,
                                     H, N if ldh is None else ldh, float(beta), int(mode), ctypes.byref(o))


def step(V, W, H, beta: float, mode="joint", *, precision="fp32", kappa: float = 0.0, normalize: bool = True,
         exponent="mm", inner_iters: int = 1, gram: bool = False, objective_out=None, stream=None,
         ctx: Optional[Context] = None):
    """One outer iteration in place on W and H (see nmf_beta_step).

    ``gram``: at beta = 2, the Gram-form denominators of Table 2 (K x K products).

    ``exponent``: "mm" (gamma(beta)) or "one" (gamma = 1 for every beta).
    ``inner_iters``: sub-iterations L (Algorithm 1 or 2; joint mode with L > 1
    needs float32 products and F N <= 2^28).
    ``objective_out``: optional float64 device tensor (1 element) receiving the
    objective at the entry iterate.
    """
    m = MODES.get(mode, mode) if isinstance(mode, str) else int(mode)
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    F, N = V.shape
    K = W.shape[1]
    if W.shape[0] != F or H.shape != (K, N):
        raise ValueError("shape mismatch: V (F,N), W (F,K), H (K,N)")
    o = _opts(precision, kappa, inner_iters, normalize, exponent, gram)
    pobj = _dev_f64(objective_out, "objective_out") if objective_out is not None else None
    st = lib().nmf_beta_step(_ctx(ctx), _stream(stream), F, N, K, pv, ldv, pw, ldw, ph, ldh,
                             float(beta), m, ctypes.byref(o), pobj)
    _check(st, "nmf_beta_step")


def step_noalloc(V, W, H, beta: float, mode="joint", *, precision="fp32", kappa: float = 0.0,
                 normalize: bool = True, exponent="mm", inner_iters: int = 1, objective_out=None, flags_out=None,
                 stream=None, ctx: Optional[Context] = None):
    """step() without any device allocation (nmf_beta_step_noalloc): the
    library's fixed per-GPU scratch array is the workspace.  ``flags_out``:
    optional int32 device tensor (1 entry) into which the step's sticky flag
    bits are OR-ed.  Raises NmfError (NMF_ERR_WORKSPACE) when the step does
    not fit in the scratch array."""
    import torch
    m = MODES.get(mode, mode) if isinstance(mode, str) else int(mode)
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    F, N = V.shape
    K = W.shape[1]
    if W.shape[0] != F or H.shape != (K, N):
        raise ValueError("shape mismatch: V (F,N), W (F,K), H (K,N)")
    o = _opts(precision, kappa, inner_iters, normalize, exponent)
    pobj = _dev_f64(objective_out, "objective_out") if objective_out is not None else None
    pfl = None
    if flags_out is not None:
        if flags_out.dtype != torch.int32 or not flags_out.is_cuda or flags_out.numel() < 1:
            raise ValueError("flags_out must be an int32 device tensor with at least 1 entry")
        pfl = flags_out.data_ptr()
    st = lib().nmf_beta_step_noalloc(_ctx(ctx), _stream(stream), F, N, K, pv, ldv, pw, ldw, ph, ldh,
                                     float(beta), m, ctypes.byref(o), pobj, pfl)
    _check(st, "nmf_beta_step_noalloc")


def objective(V, W, H, beta: float, *, kappa: float = 0.0, out=None, stream=None, ctx=None):
    """D_beta(V + kappa | WH + kappa) as a 1-element float64 device tensor."""
    import torch
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=V.device)
    st = lib().nmf_beta_objective(_ctx(ctx), _stream(stream), V.shape[0], V.shape[1], W.shape[1],
                                  pv, ldv, pw, ldw, ph, ldh, float(beta), float(kappa), out.data_ptr())
    _check(st, "nmf_beta_objective")
    return out


def grad(V, W, H, beta: float, *, kappa: float = 0.0, scale: float = 1.0, scale_dev=None, dW=None, dH=None,
         objective_out=None, stream=None, ctx=None):
    """(dW, dH) = scale * gradient of D_beta w.r.t. (W, H); see nmf_beta_grad.

    ``scale_dev``: optional float64 device tensor (1 entry) multiplying the
    gradient as well, read on the device (no host synchronization)."""
    import torch
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    if dW is None:
        dW = torch.empty_like(W)
    if dH is None:
        dH = torch.empty_like(H)
    pdw, lddw = _mat(dW, "dW")
    pdh, lddh = _mat(dH, "dH")
    pobj = _dev_f64(objective_out, "objective_out") if objective_out is not None else None
    psc = _dev_f64(scale_dev, "scale_dev") if scale_dev is not None else None
    st = lib().nmf_beta_grad(_ctx(ctx), _stream(stream), V.shape[0], V.shape[1], W.shape[1], pv, ldv, pw, ldw,
                             ph, ldh, float(beta), float(kappa), float(scale), psc, pdw, lddw, pdh, lddh, pobj)
    _check(st, "nmf_beta_grad")
    return dW, dH


def kkt(V, W, H, beta: float, *, kappa: float = 0.0, out=None, stream=None, ctx=None):
    """KKT residuals (res(W), res(H)) of Sec. 4.1.5 as a 2-element float64 device tensor."""
    import torch
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=V.device)
    st = lib().nmf_beta_kkt(_ctx(ctx), _stream(stream), V.shape[0], V.shape[1], W.shape[1], pv, ldv, pw, ldw,
                            ph, ldh, float(beta), float(kappa), _dev_f64(out, "out", 2))
    _check(st, "nmf_beta_kkt")
    return out


def run(V, W, H, beta: float, mode="joint", max_iters: int = 1000, eps: float = 1e-5, *, precision="fp32",
        kappa: float = 0.0, normalize: bool = True, exponent="mm", inner_iters: int = 1, gram: bool = False,
        trace=None, stop=None, stream=None, ctx: Optional[Context] = None):
    """Up to max_iters outer iterations with the stopping rule of Sec. 4.1.2 on
    the device (nmf_beta_run).  Returns (trace, stop): a float64 device tensor of
    max_iters + 1 objectives (entries after the stop are left as given) and an
    int32 device tensor holding the stop iteration or -1."""
    import torch
    m = MODES.get(mode, mode) if isinstance(mode, str) else int(mode)
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    F, N = V.shape
    K = W.shape[1]
    if W.shape[0] != F or H.shape != (K, N):
        raise ValueError("shape mismatch: V (F,N), W (F,K), H (K,N)")
    if trace is None:
        trace = torch.full((int(max_iters) + 1,), float("nan"), dtype=torch.float64, device=V.device)
    if stop is None:
        stop = torch.empty(1, dtype=torch.int32, device=V.device)
    if stop.dtype != torch.int32 or not stop.is_cuda or stop.numel() < 1:
        raise ValueError("stop must be an int32 device tensor")
    o = _opts(precision, kappa, inner_iters, normalize, exponent, gram)
    st = lib().nmf_beta_run(_ctx(ctx), _stream(stream), F, N, K, pv, ldv, pw, ldw, ph, ldh, float(beta), m,
                            ctypes.byref(o), int(max_iters), float(eps), _dev_f64(trace, "trace", int(max_iters) + 1),
                            stop.data_ptr())
    _check(st, "nmf_beta_run")
    return trace, stop


def validate(V, W, H, beta: float, *, kappa: float = 0.0, stream=None, ctx=None):
    pv, ldv = _mat(V, "V")
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    st = lib().nmf_beta_validate(_ctx(ctx), _stream(stream), V.shape[0], V.shape[1], W.shape[1],
                                 pv, ldv, pw, ldw, ph, ldh, float(beta), float(kappa))
    _check(st, "nmf_beta_validate")


def get_flags(clear: bool = False, stream=None, ctx=None) -> int:
    f = _u32()
    _check(lib().nmf_get_flags(_ctx(ctx), _stream(stream), ctypes.byref(f), 1 if clear else 0), "nmf_get_flags")
    return int(f.value)


def _make_autograd():
    import torch

    class BetaDivergence(torch.autograd.Function):
        """D_beta(V + kappa | WH + kappa) with a GPU backward w.r.t. W and H.

        forward(V, W, H, beta, kappa) returns a 0-d float64 tensor; the backward
        calls nmf_beta_grad with the incoming gradient as a device scale (no
        host synchronization, so the backward can be captured in a graph).  No
        gradient is returned for V, beta or kappa.
        """

        @staticmethod
        def forward(ctx_, V, W, H, beta, kappa=0.0):
            Wc, Hc = W.detach().contiguous(), H.detach().contiguous()
            out = objective(V.detach().contiguous(), Wc, Hc, beta, kappa=kappa)
            ctx_.save_for_backward(V, W, H)
            ctx_.beta = float(beta)
            ctx_.kappa = float(kappa)
            return out.reshape(())

        @staticmethod
        def backward(ctx_, g):
            V, W, H = ctx_.saved_tensors
            gd = g.detach().reshape(1).to(device=W.device, dtype=torch.float64).contiguous()
            dW, dH = grad(V.detach().contiguous(), W.detach().contiguous(), H.detach().contiguous(),
                          ctx_.beta, kappa=ctx_.kappa, scale_dev=gd)
            return None, dW.to(W.dtype), dH.to(H.dtype), None, None

    return BetaDivergence


class _LazyAutograd:
    _cls = None

    def __getattr__(self, item):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, item)


BetaDivergence = _LazyAutograd()


def beta_divergence(V, W, H, beta: float, kappa: float = 0.0):
    """Differentiable D_beta(V + kappa | WH + kappa) (float64 0-d tensor)."""
    return BetaDivergence.apply(V, W, H, beta, kappa)


# ---------------------------------------------------------------------------
# beta = 1 with a sparse V
# ---------------------------------------------------------------------------
class SparseV:
    """V (F x N) by its nonzero entries in row order (CSR) and column order (CSC),
    as device tensors: row_ptr int64 [F + 1], col_idx int32 [nnz], row_val float32
    [nnz], col_ptr int64 [N + 1], row_idx int32 [nnz], col_val float32 [nnz]."""

    def __init__(self, F, N, row_ptr, col_idx, row_val, col_ptr, row_idx, col_val):
        import torch
        self.F, self.N = int(F), int(N)
        self.nnz = int(col_idx.numel())
        spec = [("row_ptr", row_ptr, torch.int64, self.F + 1), ("col_idx", col_idx, torch.int32, self.nnz),
                ("row_val", row_val, torch.float32, self.nnz), ("col_ptr", col_ptr, torch.int64, self.N + 1),
                ("row_idx", row_idx, torch.int32, self.nnz), ("col_val", col_val, torch.float32, self.nnz)]
        for name, t, dt, n in spec:
            if not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_cuda or t.numel() != n \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {dt} device tensor with {n} entries")
            setattr(self, name, t)

    @classmethod
    def from_dense(cls, V):
        """Both compressed orders of a dense V (device or host tensor / array)."""
        import torch
        V = torch.as_tensor(V)
        dev = V.device if V.is_cuda else torch.device("cuda", torch.cuda.current_device())
        V = V.to(dev, torch.float32)
        F, N = V.shape

        def compress(M, lines):
            idx = torch.nonzero(M)  # row-major order: lines ascending, then positions
            ptr = torch.zeros(lines + 1, dtype=torch.int64, device=dev)
            ptr[1:] = torch.cumsum(torch.bincount(idx[:, 0], minlength=lines), 0)
            return ptr, idx[:, 1].to(torch.int32).contiguous(), M[idx[:, 0], idx[:, 1]].contiguous()

        rp, ci, rv = compress(V, F)
        cp, ri, cv = compress(V.t().contiguous(), N)
        return cls(F, N, rp, ci, rv, cp, ri, cv)

    def _struct(self):
        return _SparseV(self.F, self.N, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                        self.row_val.data_ptr(), self.col_ptr.data_ptr(), self.row_idx.data_ptr(),
                        self.col_val.data_ptr())


def kl_step_sparse(Vs: SparseV, W, H, mode="joint", *, normalize: bool = True, objective_out=None, stream=None,
                   ctx: Optional[Context] = None):
    """One outer iteration at beta = 1 on a sparse V (nmf_kl_step_sparse), in place."""
    m = MODES.get(mode, mode) if isinstance(mode, str) else int(mode)
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    K = W.shape[1]
    if W.shape[0] != Vs.F or H.shape != (K, Vs.N):
        raise ValueError("shape mismatch: W (F,K), H (K,N)")
    o = _opts(normalize=normalize)
    pobj = _dev_f64(objective_out, "objective_out") if objective_out is not None else None
    sv = Vs._struct()
    _check(lib().nmf_kl_step_sparse(_ctx(ctx), _stream(stream), ctypes.byref(sv), K, pw, ldw, ph, ldh, m,
                                    ctypes.byref(o), pobj), "nmf_kl_step_sparse")


def kl_objective_sparse(Vs: SparseV, W, H, *, out=None, stream=None, ctx=None):
    """D_1(V | WH) for a sparse V as a 1-element float64 device tensor."""
    import torch
    pw, ldw = _mat(W, "W")
    ph, ldh = _mat(H, "H")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=W.device)
    sv = Vs._struct()
    _check(lib().nmf_kl_objective_sparse(_ctx(ctx), _stream(stream), ctypes.byref(sv), W.shape[1], pw, ldw, ph,
                                         ldh, _dev_f64(out, "out")), "nmf_kl_objective_sparse")
    return out


def sparse_validate(Vs: SparseV, *, stream=None, ctx=None):
    sv = Vs._struct()
    _check(lib().nmf_sparse_validate(_ctx(ctx), _stream(stream), ctypes.byref(sv)), "nmf_sparse_validate")


# ---------------------------------------------------------------------------
# many problems in one launch
# ---------------------------------------------------------------------------
def _problems(problems):
    """[(V, W, H, beta), ...] of device tensors -> ctypes array (tensors kept alive by the caller)."""
    arr = (_Problem * len(problems))()
    for i, (V, W, H, beta) in enumerate(problems):
        v, ldv = _mat(V, "V")
        w, ldw = _mat(W, "W", True)
        h, ldh = _mat(H, "H", True)
        F, N = V.shape
        K = W.shape[1]
        if W.shape[0] != F or H.shape != (K, N):
            raise ValueError(f"problem {i}: shapes V {tuple(V.shape)}, W {tuple(W.shape)}, H {tuple(H.shape)}")
        arr[i] = _Problem(F, N, K, v, ldv, w, ldw, h, ldh, float(beta))
    return arr


class Batch:
    """Many problems updated by one persistent launch per outer iteration
    (nmf_batch_create / nmf_batch_step).  ``problems`` is a list of
    (V, W, H, beta) device tensors; W and H are updated in place by step()."""

    def __init__(self, problems, mode="joint", *, precision="fp32", kappa: float = 0.0, normalize: bool = True,
                 exponent="mm", tiles_per_item: int = 0, workers: int = 0, lag: int = 0,
                 ctx: Optional[Context] = None):
        self._tensors = list(problems)  # keep the caller's tensors alive
        self.count = len(problems)
        arr = _problems(problems)
        o = _opts(precision, kappa, 1, normalize, exponent)
        cfg = _BatchConfig(int(tiles_per_item), int(workers), int(lag))
        h = _vp()
        _check(lib().nmf_batch_create(_ctx(ctx), arr, self.count, MODES[mode], ctypes.byref(o), ctypes.byref(cfg),
                                      ctypes.byref(h)), "nmf_batch_create")
        self.handle = h

    def step(self, objectives=None, stream=None):
        """One outer iteration of every problem; ``objectives``: optional float64
        device tensor of ``count`` entries receiving the entry objectives."""
        optr = None
        if objectives is not None:
            import torch
            if objectives.dtype != torch.float64 or not objectives.is_cuda or objectives.numel() < self.count:
                raise ValueError("objectives must be a float64 device tensor with one entry per problem")
            optr = objectives.data_ptr()
        _check(lib().nmf_batch_step(self.handle, _stream(stream), optr), "nmf_batch_step")

    def flags(self, clear: bool = False, stream=None) -> int:
        f = _u32()
        _check(lib().nmf_batch_get_flags(self.handle, _stream(stream), ctypes.byref(f), 1 if clear else 0),
               "nmf_batch_get_flags")
        return int(f.value)

    def info(self):
        n, w, b = _i64(), _i32(), _i64()
        _check(lib().nmf_batch_info(self.handle, ctypes.byref(n), ctypes.byref(w), ctypes.byref(b)), "nmf_batch_info")
        return {"work_items": n.value, "workers": w.value, "device_bytes": b.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().nmf_batch_destroy(self.handle)
            self.handle = _vp()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def batch_bucket(F: int, N: int, K: int, beta: float) -> int:
    """Tile-table bucket of a batched problem of sizes F, N, K and divergence
    beta (nmf_batch_bucket)."""
    return int(lib().nmf_batch_bucket(int(F), int(N), int(K), float(beta)))


def set_batch_tiles(tiles, ctx: Optional[Context] = None):
    """Sets the context's tiles per pass item of each bucket (nmf_set_batch_tiles)."""
    if len(tiles) != BATCH_BUCKETS:
        raise ValueError(f"{BATCH_BUCKETS} tile counts expected")
    arr = (_i32 * BATCH_BUCKETS)(*[int(t) for t in tiles])
    _check(lib().nmf_set_batch_tiles(_ctx(ctx), arr), "nmf_set_batch_tiles")


def get_batch_tiles(ctx: Optional[Context] = None):
    arr = (_i32 * BATCH_BUCKETS)()
    _check(lib().nmf_get_batch_tiles(_ctx(ctx), arr), "nmf_get_batch_tiles")
    return list(arr)


def tune(problems, mode="joint", *, precision="fp32", kappa: float = 0.0, normalize: bool = True,
         iters: int = 3, cache: Optional[str] = None, stream=None, ctx: Optional[Context] = None):
    """Tunes the context's per-bucket tile table on ``problems`` (nmf_tune) and
    returns (tiles, ms per step, from_cache).  With ``cache`` (a text file) a
    table measured before for the same device, mode and precision covering
    these problems' buckets is installed without measuring; new results are
    written to the file."""
    arr = _problems(problems)
    o = _opts(precision, kappa, 1, normalize)
    tiles = (_i32 * BATCH_BUCKETS)()
    ms, hit = _dbl(), _i32()
    path = os.fsencode(cache) if cache else None
    _check(lib().nmf_tune(_ctx(ctx), _stream(stream), arr, len(problems), MODES[mode], ctypes.byref(o), int(iters),
                          path, tiles, ctypes.byref(ms), ctypes.byref(hit)), "nmf_tune")
    return list(tiles), ms.value, bool(hit.value)


def batch_requirements(shapes, mode="joint", tiles=None, precision="fp32"):
    """(work items per step, workspace bytes) that problems of the given
    (F, N, K, beta) sizes need in a batch in ``mode`` and ``precision`` under
    ``tiles`` (None: 256 in every bucket).  Host only."""
    arr = (_Problem * len(shapes))()
    for i, (F, N, K, beta) in enumerate(shapes):
        arr[i] = _Problem(int(F), int(N), int(K), None, 0, None, 0, None, 0, float(beta))
    t = (_i32 * BATCH_BUCKETS)(*[int(x) for x in tiles]) if tiles is not None else None
    n, b = _i64(), _i64()
    _check(lib().nmf_batch_requirements(arr, len(shapes), MODES[mode], PRECISIONS[precision], t, ctypes.byref(n),
                                        ctypes.byref(b)),
           "nmf_batch_requirements")
    return n.value, b.value


def reserve_batched(max_problems: int, max_items: int, workspace_bytes: int, ctx: Optional[Context] = None):
    """Allocates the context's region for step_batched (nmf_reserve_batched)."""
    _check(lib().nmf_reserve_batched(_ctx(ctx), int(max_problems), int(max_items), int(workspace_bytes)),
           "nmf_reserve_batched")


class DeviceProblems:
    """Problem descriptors (nmf_problem) in device memory for step_batched.
    ``capacity`` slots; set() writes (V, W, H, beta) device tensors into them
    with one host-to-device copy on ``stream`` (the tensors are kept alive)."""

    def __init__(self, capacity: int, device: int = 0):
        import torch
        self.capacity = int(capacity)
        self.buf = torch.zeros(ctypes.sizeof(_Problem) * self.capacity, dtype=torch.uint8,
                               device=f"cuda:{device}")
        self._tensors = []
        self.count = 0

    def set(self, problems, stream=None):
        import torch
        if len(problems) > self.capacity:
            raise ValueError(f"{len(problems)} problems for {self.capacity} slots")
        arr = _problems(problems)
        host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
        n = host.numel()
        if n:
            if stream is None:
                self.buf[:n].copy_(host)
            else:
                with torch.cuda.stream(stream):
                    self.buf[:n].copy_(host)
        self._tensors = list(problems)
        self.count = len(problems)

    def set_raw(self, descriptors: bytes, stream=None):
        """Writes packed nmf_problem bytes as they are (no checks), for tests of
        the device-side checks."""
        import torch
        host = torch.frombuffer(bytearray(descriptors), dtype=torch.uint8)
        self.buf[:host.numel()].copy_(host)

    @staticmethod
    def pack(problems) -> bytes:
        return bytes(_problems(problems))

    def ptr(self) -> int:
        return self.buf.data_ptr()


def step_batched(dp: DeviceProblems, mode="joint", *, count: Optional[int] = None, precision="fp32",
                 kappa: float = 0.0, normalize: bool = True, exponent="mm", objectives=None, d_count=None,
                 stream=None, ctx: Optional[Context] = None):
    """One outer iteration of every problem described in device memory
    (nmf_beta_step_batched).  ``count`` descriptors are passed (default: those
    set last); ``d_count`` (an int32 device tensor, optional) limits the number
    used on the device; ``objectives`` (float64 device tensor) receives the
    entry objectives."""
    import torch
    n = dp.count if count is None else int(count)
    optr = None
    if objectives is not None:
        if objectives.dtype != torch.float64 or not objectives.is_cuda or objectives.numel() < n:
            raise ValueError("objectives must be a float64 device tensor with one entry per problem")
        optr = objectives.data_ptr()
    cptr = None
    if d_count is not None:
        if d_count.dtype != torch.int32 or not d_count.is_cuda:
            raise ValueError("d_count must be an int32 device tensor")
        cptr = d_count.data_ptr()
    o = _opts(precision, kappa, 1, normalize, exponent)
    _check(lib().nmf_beta_step_batched(_ctx(ctx), _stream(stream), n, dp.ptr(), MODES[mode], ctypes.byref(o), optr,
                                       cptr), "nmf_beta_step_batched")
