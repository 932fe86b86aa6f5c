"""Python binding of the gfx950 ILS splitting solver (libils.so).

Argument marshalling only: every step of every method runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  The
library must have been built (``build.build()``); importing this package
never falls back to any other implementation, and calls fail loudly if the
library or a GPU is missing.

Matrices are column-major: pass A as an (m, n) float64 CUDA tensor with
strides (1, lda), e.g. ``torch.empty(n, lda, dtype=torch.float64,
device='cuda').t()[:m]`` or ``ils.fortran(A)``.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

from . import build as _build

OK, ERR_ARG, ERR_NOT_SPD, ERR_NO_CONVERGENCE, ERR_NONFINITE, ERR_HIP, ERR_ALLOC = 0, -1, -2, -3, -4, -5, -6
STOP_RR, STOP_XREF, STOP_FIXED = 0, 1, 2
FORM_PAPER, FORM_CORRECTION = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
SAMPLE_UNIFORM, SAMPLE_NORM = 0, 1
GRAM_SPLITK, GRAM_PERSISTENT = 0, 1
BATCH_LARGEST_FIRST, BATCH_AS_GIVEN = 0, 1
RESID_AUTO, RESID_TWO_PASS = 0, 1

LIB_PATH = _build.LIB
EXPORTS = ("ils_create", "ils_destroy", "ils_opts_default", "ils_status_string", "ils_sp_solve",
           "ils_rk_solve", "ils_rgs_solve", "ils_gram", "ils_colpass", "ils_residual", "ils_residual_noalloc",
           "ils_spd_solve", "ils_rk_indices", "ils_scd_subsets", "ils_set_profiling",
           "ils_get_phase_times", "ils_sp_solve_batched", "ils_sp_solve_multi", "ils_rk_solve_multi", "ils_sp_prepare",
           "ils_sp_prep_solve_multi", "ils_sp_prep_destroy", "ils_atjb", "ils_ws_create",
           "ils_ws_destroy", "ils_ws_train", "ils_ws_infer", "ils_ws_save", "ils_ws_load",
           "ils_ws_nparams", "ils_ws_get_params", "ils_ws_set_params", "ils_ws_forward", "ils_ws_grad",
           "ils_ws_adam", "ils_csr_create", "ils_csr_destroy", "ils_sp_solve_csr", "ils_rk_solve_csr",
           "ils_rgs_solve_csr", "ils_csr_gram", "ils_csr_colpass", "ils_csr_residual",
           "ils_csr_export_csc", "ils_tune_gram", "ils_tune_batched", "ils_tune_residual", "ils_tune_save", "ils_tune_load", "ils_tune_clear")
PHASES = ("colpass", "gram", "gram_reduce", "rhs", "gauss_jordan", "layout", "iterations")


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("stop_rule", C.c_int32), ("form", C.c_int32),
                ("precision", C.c_int32), ("sampling", C.c_int32), ("x_ref", C.c_void_p),
                ("max_outer", C.c_int64), ("max_inner", C.c_int64), ("inner_tol", C.c_double),
                ("inner_check", C.c_int64), ("seed", C.c_uint64), ("stream_offset", C.c_uint64),
                ("alpha", C.c_int64)]


class Problem(C.Structure):
    _fields_ = [("p", C.c_int64), ("q", C.c_int64), ("n", C.c_int64), ("lda", C.c_int64),
                ("A", C.c_void_p), ("b", C.c_void_p), ("x0", C.c_void_p), ("x_ref", C.c_void_p),
                ("x", C.c_void_p)]


class _Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("pad", C.c_int32), ("outer_iters", C.c_int64),
                ("inner_iters", C.c_int64), ("rr", C.c_double), ("rel_err", C.c_double),
                ("device_ms", C.c_double)]


@dataclasses.dataclass
class Info:
    status: int
    outer_iters: int
    inner_iters: int
    rr: float
    rel_err: float
    device_ms: float


class ILSError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libils.so and declare the C ABI.  Raises if the file is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ILSError(f"{path} is missing: build it with paper_2203_15340_amd.build.build()")
    L = C.CDLL(path)
    P, I64, U64, I32 = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32
    solve_args = [P, I64, I64, I64, P, I64, P, P, P, P, P]
    sig = {
        "ils_create": (C.c_int, [C.POINTER(P), C.c_int, P]),
        "ils_destroy": (C.c_int, [P]),
        "ils_opts_default": (None, [P]),
        "ils_status_string": (C.c_char_p, [C.c_int]),
        "ils_sp_solve": (C.c_int, solve_args),
        "ils_rk_solve": (C.c_int, solve_args),
        "ils_rgs_solve": (C.c_int, solve_args),
        "ils_gram": (C.c_int, [P, I64, I64, I64, P, I64, P, I64, I32]),
        "ils_colpass": (C.c_int, [P, I64, I64, I64, P, I64, P, P, P]),
        "ils_residual": (C.c_int, [P, I64, I64, I64, P, I64, P, P, P]),
        "ils_residual_noalloc": (C.c_int, [P, I64, I64, I64, P, I64, P, P, P]),
        "ils_spd_solve": (C.c_int, [P, I64, I64, P, I64, P, I64, P, I64]),
        "ils_rk_indices": (C.c_int, [P, U64, U64, I64, I64, P, I64, P, P]),
        "ils_scd_subsets": (C.c_int, [P, U64, U64, I64, I64, I64, I64, P, P]),
        "ils_set_profiling": (C.c_int, [P, C.c_int]),
        "ils_sp_solve_batched": (C.c_int, [P, I64, P, P, P]),
        "ils_get_phase_times": (C.c_int, [P, P, C.c_int]),
        "ils_sp_solve_multi": (C.c_int, [P, I64, I64, I64, P, I64, I64, P, I64, P, I64, P, I64, P,
                                         P, P]),
        "ils_rk_solve_multi": (C.c_int, [P, I64, I64, I64, P, I64, I64, P, I64, P, I64, P, I64, P,
                                         P, P]),
        "ils_sp_prepare": (C.c_int, [P, I64, I64, I64, P, I64, C.POINTER(P)]),
        "ils_sp_prep_solve_multi": (C.c_int, [P, I64, P, I64, P, I64, P, I64, P, P, P]),
        "ils_sp_prep_destroy": (C.c_int, [P]),
        "ils_atjb": (C.c_int, [P, I64, I64, I64, P, I64, I64, P, I64, P, I64]),
        "ils_ws_create": (C.c_int, [P, I64, I64, I64, P, I64, U64, C.POINTER(P)]),
        "ils_ws_destroy": (C.c_int, [P]),
        "ils_ws_train": (C.c_int, [P, I64, P, I64, P, I64, I32, I64, C.c_double, P]),
        "ils_ws_infer": (C.c_int, [P, I64, P, I64, P, I64]),
        "ils_ws_save": (C.c_int, [P, C.c_char_p]),
        "ils_ws_load": (C.c_int, [P, C.c_char_p]),
        "ils_ws_nparams": (C.c_int, [P, P]),
        "ils_ws_get_params": (C.c_int, [P, P]),
        "ils_ws_set_params": (C.c_int, [P, P]),
        "ils_ws_forward": (C.c_int, [P, I64, P, P]),
        "ils_ws_grad": (C.c_int, [P, I64, P, P, P, P]),
        "ils_ws_adam": (C.c_int, [P, P, C.c_double]),
        "ils_csr_create": (C.c_int, [P, I64, I64, I64, I64, P, P, P, C.POINTER(P)]),
        "ils_csr_destroy": (C.c_int, [P]),
        "ils_sp_solve_csr": (C.c_int, [P, P, P, P, P, P, P]),
        "ils_rk_solve_csr": (C.c_int, [P, P, P, P, P, P, P]),
        "ils_rgs_solve_csr": (C.c_int, [P, P, P, P, P, P, P]),
        "ils_csr_gram": (C.c_int, [P, P, I32, P, I64]),
        "ils_csr_colpass": (C.c_int, [P, P, P, P, P]),
        "ils_csr_residual": (C.c_int, [P, P, P, P, P]),
        "ils_csr_export_csc": (C.c_int, [P, P, P, P, P]),
        "ils_tune_gram": (C.c_int, [P, I64, I64, P, I64, I32, I32, P]),
        "ils_tune_batched": (C.c_int, [P, I64, P, P, I32, P]),
        "ils_tune_residual": (C.c_int, [P, I64, I64, I64, P, I64, P, P, I32, P]),
        "ils_tune_save": (C.c_int, [C.c_char_p]),
        "ils_tune_load": (C.c_int, [C.c_char_p]),
        "ils_tune_clear": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(code: int) -> str:
    return load_library().ils_status_string(code).decode()


def _torch():
    import torch
    return torch


_handles = {}


def handle(device=None):
    """Library handle bound to `device` and torch's current stream there."""
    torch = _torch()
    dev = None
    if device is not None:
        dev = device.index if isinstance(device, torch.device) else torch.device(device).index
    if dev is not None and _handles:
        # repeated calls: the raw current stream and one lookup (host time
        # here is time the device waits for the first kernel of a solve)
        h = _handles.get((dev, torch._C._cuda_getCurrentRawStream(dev)))
        if h is not None:
            return h
    if not torch.cuda.is_available():
        raise ILSError("no GPU visible: the ILS library runs only on the GPU")
    if dev is None:
        dev = torch.cuda.current_device()
    stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, stream)
    if key not in _handles:
        h = C.c_void_p()
        rc = load_library().ils_create(C.byref(h), dev, C.c_void_p(stream))
        if rc != OK:
            raise ILSError(f"ils_create failed: {status_string(rc)}")
        _handles[key] = h
    return _handles[key]


def fortran(A):
    """Column-major copy (or view) of a 2-D tensor: strides (1, m)."""
    if A.dim() == 2 and A.stride(0) == 1 and A.stride(1) >= max(1, A.shape[0]):
        return A
    return A.t().contiguous().t()


def _ld(M):
    """Leading dimension of a column-major 2-D tensor (strides (1, ld))."""
    if M.dim() != 2 or (M.shape[0] > 1 and M.stride(0) != 1):
        raise ILSError("matrices must be column-major: strides (1, ld)")
    return M.stride(1) if M.shape[1] > 1 else max(1, M.shape[0])


def _check_vec(v, n, name):
    if v is None:
        return None
    if not v.is_cuda or v.dtype != _torch().float64 or v.numel() != n or not v.is_contiguous():
        raise ILSError(f"{name} must be a contiguous float64 CUDA tensor with {n} entries")
    return v


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


_opts_default = None


def make_opts(tol=1e-6, stop_rule=STOP_RR, form=FORM_PAPER, precision=PREC_FP64,
              sampling=SAMPLE_UNIFORM, x_ref=None, max_outer=20000, max_inner=-1, inner_tol=-1.0,
              inner_check=-1, seed=0, stream_offset=0, alpha=0):
    global _opts_default
    if _opts_default is None:
        d = Opts()
        load_library().ils_opts_default(C.byref(d))
        _opts_default = bytes(d)
    o = Opts.from_buffer_copy(_opts_default)
    o.tol, o.stop_rule, o.form, o.precision, o.sampling = tol, stop_rule, form, precision, sampling
    o.x_ref = None if x_ref is None else x_ref.data_ptr()
    o.max_outer, o.max_inner, o.inner_tol, o.inner_check = max_outer, max_inner, inner_tol, inner_check
    o.seed, o.stream_offset, o.alpha = seed, stream_offset, alpha
    return o


def _solve(fname, A, b, p, x0=None, out=None, raise_on_error=False, **kw):
    torch = _torch()
    if A.dim() != 2 or A.dtype != torch.float64 or not A.is_cuda:
        raise ILSError("A must be a column-major (stride (1, lda)) float64 CUDA tensor")
    m, n = A.shape
    lda = _ld(A)
    _check_vec(b, m, "b")
    _check_vec(x0, n, "x0")
    x_ref = _check_vec(kw.get("x_ref"), n, "x_ref")
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    _check_vec(x, n, "out")
    o = make_opts(**kw)
    info = _Info()
    h = handle(A.device)
    rc = getattr(load_library(), fname)(h, p, m - p, n, _ptr(A), lda, _ptr(b), _ptr(x0), _ptr(x),
                                        C.byref(o), C.byref(info))
    del x_ref
    res = Info(int(rc), int(info.outer_iters), int(info.inner_iters), float(info.rr),
               float(info.rel_err), float(info.device_ms))
    if raise_on_error and rc != OK:
        raise ILSError(f"{fname}: {status_string(rc)}")
    return x, res


def sp_solve(A, b, p, x0=None, **kw):
    """SP method (Algorithm 1).  Returns (x, Info)."""
    return _solve("ils_sp_solve", A, b, p, x0, **kw)


def _check_mat(M, rows, cols, name):
    torch = _torch()
    if M is None:
        return None
    if M.dim() != 2 or M.dtype != torch.float64 or not M.is_cuda or tuple(M.shape) != (rows, cols) \
            or (cols > 1 and M.stride(0) != 1):
        raise ILSError(f"{name} must be a column-major float64 CUDA tensor of shape ({rows}, {cols})")
    return M


def sp_solve_multi(A, B, p, X0=None, out=None, raise_on_error=False, **kw):
    """SP for the columns of B (m x nrhs) sharing A.  x_ref, when given, is
    an (n, nrhs) tensor with leading dimension n.  Returns (X, Info, iters)
    with iters a numpy int64 array of per-column outer counts."""
    import numpy as np
    torch = _torch()
    if A.dim() != 2 or A.dtype != torch.float64 or not A.is_cuda:
        raise ILSError("A must be a column-major (stride (1, lda)) float64 CUDA tensor")
    m, n = A.shape
    nrhs = B.shape[1]
    _check_mat(B, m, nrhs, "B")
    _check_mat(X0, n, nrhs, "X0")
    xr = kw.get("x_ref")
    if xr is not None:
        _check_mat(xr, n, nrhs, "x_ref")
        if nrhs > 1 and xr.stride(1) != n:
            raise ILSError("x_ref must have leading dimension n")
    X = out if out is not None else torch.empty((nrhs, n), dtype=torch.float64, device=A.device).t()
    _check_mat(X, n, nrhs, "out")
    o = make_opts(**kw)
    info = _Info()
    iters = np.zeros(nrhs, dtype=np.int64)
    rc = load_library().ils_sp_solve_multi(
        handle(A.device), p, m - p, n, _ptr(A), _ld(A), nrhs, _ptr(B), _ld(B), _ptr(X0),
        n if X0 is None else _ld(X0), _ptr(X), _ld(X), C.byref(o), iters.ctypes.data, C.byref(info))
    res = Info(int(rc), int(info.outer_iters), int(info.inner_iters), float(info.rr),
               float(info.rel_err), float(info.device_ms))
    if raise_on_error and rc != OK:
        raise ILSError(f"ils_sp_solve_multi: {status_string(rc)}")
    return X, res, iters


class SPPrepared:
    """SP on a fixed A (ils_sp_prepare): the Gram products and the
    elimination are done here once; solve_multi then costs A^T J B, one
    product with P and the outer steps.  A (column-major float64 CUDA
    tensor) must stay alive and unchanged while this object lives."""

    def __init__(self, A, p):
        torch = _torch()
        if A.dim() != 2 or A.dtype != torch.float64 or not A.is_cuda:
            raise ILSError("A must be a column-major (stride (1, lda)) float64 CUDA tensor")
        self.A = A
        self.m, self.n = A.shape
        self.p = p
        self._h = handle(A.device)
        obj = C.c_void_p()
        _rc(load_library().ils_sp_prepare(self._h, p, self.m - p, self.n, _ptr(A), _ld(A), C.byref(obj)),
            "ils_sp_prepare")
        self._obj = obj

    def close(self):
        if getattr(self, "_obj", None):
            load_library().ils_sp_prep_destroy(self._obj)
            self._obj = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve_multi(self, B, X0=None, out=None, raise_on_error=False, **kw):
        """As sp_solve_multi.  Returns (X, Info, iters)."""
        import numpy as np
        torch = _torch()
        nrhs = B.shape[1]
        _check_mat(B, self.m, nrhs, "B")
        _check_mat(X0, self.n, nrhs, "X0")
        xr = kw.get("x_ref")
        if xr is not None:
            _check_mat(xr, self.n, nrhs, "x_ref")
            if nrhs > 1 and xr.stride(1) != self.n:
                raise ILSError("x_ref must have leading dimension n")
        X = out if out is not None else torch.empty((nrhs, self.n), dtype=torch.float64,
                                                    device=self.A.device).t()
        _check_mat(X, self.n, nrhs, "out")
        o = make_opts(**kw)
        info = _Info()
        iters = np.zeros(nrhs, dtype=np.int64)
        rc = load_library().ils_sp_prep_solve_multi(
            self._obj, nrhs, _ptr(B), _ld(B), _ptr(X0), self.n if X0 is None else _ld(X0), _ptr(X), _ld(X),
            C.byref(o), iters.ctypes.data, C.byref(info))
        res = Info(int(rc), int(info.outer_iters), int(info.inner_iters), float(info.rr),
                   float(info.rel_err), float(info.device_ms))
        if raise_on_error and rc != OK:
            raise ILSError(f"ils_sp_prep_solve_multi: {status_string(rc)}")
        return X, res, iters


def rk_solve_multi(A, B, p, X0=None, out=None, raise_on_error=False, **kw):
    """SP-RK-RGS for the columns of B (m x nrhs) sharing A and one index
    stream (column r follows rk_solve on b_r with the same seed).  x_ref,
    when given, is an (n, nrhs) tensor with leading dimension n.  Returns
    (X, Info, iters)."""
    import numpy as np
    torch = _torch()
    if A.dim() != 2 or A.dtype != torch.float64 or not A.is_cuda:
        raise ILSError("A must be a column-major (stride (1, lda)) float64 CUDA tensor")
    m, n = A.shape
    nrhs = B.shape[1]
    _check_mat(B, m, nrhs, "B")
    _check_mat(X0, n, nrhs, "X0")
    xr = kw.get("x_ref")
    if xr is not None:
        _check_mat(xr, n, nrhs, "x_ref")
        if nrhs > 1 and xr.stride(1) != n:
            raise ILSError("x_ref must have leading dimension n")
    X = out if out is not None else torch.empty((nrhs, n), dtype=torch.float64, device=A.device).t()
    _check_mat(X, n, nrhs, "out")
    o = make_opts(**kw)
    info = _Info()
    iters = np.zeros(nrhs, dtype=np.int64)
    rc = load_library().ils_rk_solve_multi(
        handle(A.device), p, m - p, n, _ptr(A), _ld(A), nrhs, _ptr(B), _ld(B), _ptr(X0),
        n if X0 is None else _ld(X0), _ptr(X), _ld(X), C.byref(o), iters.ctypes.data, C.byref(info))
    res = Info(int(rc), int(info.outer_iters), int(info.inner_iters), float(info.rr),
               float(info.rel_err), float(info.device_ms))
    if raise_on_error and rc != OK:
        raise ILSError(f"ils_rk_solve_multi: {status_string(rc)}")
    return X, res, iters


def rk_solve(A, b, p, x0=None, **kw):
    """SP-RK-RGS (Algorithm 2).  Returns (x, Info)."""
    return _solve("ils_rk_solve", A, b, p, x0, **kw)


def rgs_solve(A, b, p, x0=None, **kw):
    """SP-SCD (Algorithm 5); alpha=1 with sampling=SAMPLE_NORM is SP-RCD."""
    return _solve("ils_rgs_solve", A, b, p, x0, **kw)


def _rc(rc, what):
    if rc != OK:
        raise ILSError(f"{what}: {status_string(rc)}")


def gram(A, r0, r1, precision=PREC_FP64):
    """A[r0:r1]^T A[r0:r1] as an (n, n) column-major float64 tensor."""
    torch = _torch()
    m, n = A.shape
    G = torch.empty(n, n, dtype=torch.float64, device=A.device).t()
    _rc(load_library().ils_gram(handle(A.device), r0, r1, n, _ptr(A), _ld(A), _ptr(G), n,
                                precision), "ils_gram")
    return G


def atjb(A, B, p):
    """A^T J B (n x nrhs, column-major float64) for the columns of B."""
    torch = _torch()
    m, n = A.shape
    nrhs = B.shape[1]
    G = torch.empty((nrhs, n), dtype=torch.float64, device=A.device).t()
    _rc(load_library().ils_atjb(handle(A.device), p, m - p, n, _ptr(A), _ld(A), nrhs, _ptr(B), _ld(B),
                                _ptr(G), n), "ils_atjb")
    return G


def colpass(A, b, p):
    torch = _torch()
    m, n = A.shape
    g = torch.empty(n, dtype=torch.float64, device=A.device)
    c = torch.empty(n, dtype=torch.float64, device=A.device)
    rc = load_library().ils_colpass(handle(A.device), p, m - p, n, _ptr(A), _ld(A), _ptr(b),
                                    _ptr(g), _ptr(c))
    return rc, g, c


def residual(A, b, p, x):
    torch = _torch()
    m, n = A.shape
    r = torch.empty(n, dtype=torch.float64, device=A.device)
    _rc(load_library().ils_residual(handle(A.device), p, m - p, n, _ptr(A), _ld(A), _ptr(b),
                                    _ptr(x), _ptr(r)), "ils_residual")
    return r


def residual_noalloc(A, b, p, x, out=None):
    """r = A^T J (b - A x) through ils_residual_noalloc: the library's fixed
    device workspace, nothing allocated by the call.  Queued on torch's
    current stream; r is ready once that stream's work is done."""
    torch = _torch()
    m, n = A.shape
    r = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    _rc(load_library().ils_residual_noalloc(handle(A.device), p, m - p, n, _ptr(A), _ld(A), _ptr(b),
                                            _ptr(x), _ptr(r)), "ils_residual_noalloc")
    return r


def spd_solve(G, R):
    """G^{-1} R by block Gauss-Jordan; returns (status, X)."""
    torch = _torch()
    n = G.shape[0]
    nrhs = R.shape[1]
    X = torch.empty(nrhs, n, dtype=torch.float64, device=G.device).t()
    rc = load_library().ils_spd_solve(handle(G.device), n, nrhs, _ptr(G), _ld(G), _ptr(R),
                                      _ld(R), _ptr(X), n)
    return rc, X


def rk_indices(seed, outer, t0, count, weights):
    torch = _torch()
    j1 = torch.empty(count, dtype=torch.int32, device=weights.device)
    j2 = torch.empty(count, dtype=torch.int32, device=weights.device)
    _rc(load_library().ils_rk_indices(handle(weights.device), seed, outer, t0, count, _ptr(weights),
                                      weights.numel(), _ptr(j1), _ptr(j2)), "ils_rk_indices")
    return j1, j2


def scd_subsets(seed, outer, t0, count, n, alpha_opt=0, device="cuda"):
    torch = _torch()
    words = (n + 31) // 32
    alpha = torch.empty(count, dtype=torch.int32, device=device)
    mask = torch.empty(count, words, dtype=torch.int32, device=device)
    _rc(load_library().ils_scd_subsets(handle(device), seed, outer, t0, count, n, alpha_opt,
                                       _ptr(alpha), _ptr(mask)), "ils_scd_subsets")
    return alpha, mask


PROFILE_OFF, PROFILE_PHASES, PROFILE_GRAM = 0, 1, 2


def set_profiling(mode=PROFILE_PHASES, device=None):
    """Phase events of sp_solve: PROFILE_PHASES (every phase), PROFILE_GRAM
    (the main Gram kernel only, the cheap one to leave on while timing) or
    PROFILE_OFF; True / False mean PROFILE_PHASES / PROFILE_OFF."""
    if mode is True or mode is False:
        mode = PROFILE_PHASES if mode else PROFILE_OFF
    _rc(load_library().ils_set_profiling(handle(device), int(mode)), "ils_set_profiling")


def phase_times(device=None):
    """Phase durations (ms) of the last profiled sp_solve, keyed by PHASES
    (NaN for the phases PROFILE_GRAM does not time)."""
    buf = (C.c_double * len(PHASES))()
    n = load_library().ils_get_phase_times(handle(device), buf, len(PHASES))
    if n < 0:
        raise ILSError(f"ils_get_phase_times: {status_string(n)}")
    return dict(zip(PHASES, list(buf)[:n]))


class BatchPlan:
    """Descriptors of a batch built once (ctypes array + the tensors it points
    to), so that repeated solves cost one library call."""

    def __init__(self, problems, x_refs=None, x0s=None, outs=None):
        torch = _torch()
        nb = len(problems)
        self.arr = (Problem * nb)()
        self.xs, self._keep = [], []
        for i, (A, b, p) in enumerate(problems):
            m, n = A.shape
            x = outs[i] if outs is not None else torch.empty(n, dtype=torch.float64, device=A.device)
            xr = x_refs[i] if x_refs is not None else None
            x0 = x0s[i] if x0s is not None else None
            self.arr[i] = Problem(p, m - p, n, _ld(A), A.data_ptr(), b.data_ptr(),
                                  None if x0 is None else x0.data_ptr(),
                                  None if xr is None else xr.data_ptr(), x.data_ptr())
            self.xs.append(x)
            self._keep.append((A, b, x0, xr))
        self.device = problems[0][0].device
        self.infos = (_Info * nb)()

    def solve(self, **kw):
        o = make_opts(**kw)
        rc = load_library().ils_sp_solve_batched(handle(self.device), len(self.xs), self.arr,
                                                 C.byref(o), self.infos)
        return int(rc)

    def results(self):
        return [Info(int(f.status), int(f.outer_iters), int(f.inner_iters), float(f.rr),
                     float(f.rel_err), float(f.device_ms)) for f in self.infos]


def sp_solve_batched(problems, x_refs=None, x0s=None, outs=None, **kw):
    """SP on many problems in one launch.  problems: list of (A, b, p) with A a
    column-major float64 CUDA tensor.  Returns (list of x, list of Info, rc)."""
    plan = BatchPlan(problems, x_refs, x0s, outs)
    rc = plan.solve(**kw)
    return plan.xs, plan.results(), rc


class WarmStart:
    """The learned warm start (ils_ws_*): a BF16 perceptron mapping rows
    `in_rows` of b to an initial x for SP.  Arrays are CUDA tensors."""

    def __init__(self, m, n, in_rows, hidden=512, seed=0, device=None):
        import numpy as np
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.m, self.n = m, n
        rows = np.ascontiguousarray(in_rows, dtype=np.int64)
        self.d_in, self.hidden = len(rows), hidden
        self._h = handle(self.device)
        net = C.c_void_p()
        _rc(load_library().ils_ws_create(self._h, m, n, len(rows), rows.ctypes.data, hidden, seed,
                                         C.byref(net)), "ils_ws_create")
        self._net = net
        np_ = C.c_int64()
        _rc(load_library().ils_ws_nparams(self._net, C.byref(np_)), "ils_ws_nparams")
        self.nparams = int(np_.value)

    def close(self):
        if self._net:
            load_library().ils_ws_destroy(self._net)
            self._net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train(self, B, X, epochs=10, batch=256, lr=1e-3):
        """B: (m, N), X: (n, N) column-major float64.  Returns the last epoch's mean loss."""
        loss = C.c_double()
        _rc(load_library().ils_ws_train(self._net, B.shape[1], _ptr(B), _ld(B), _ptr(X), _ld(X),
                                        epochs, batch, lr, C.byref(loss)), "ils_ws_train")
        return float(loss.value)

    def infer(self, B, out=None):
        torch = _torch()
        N = B.shape[1]
        X0 = out if out is not None else torch.empty((N, self.n), dtype=torch.float64,
                                                     device=B.device).t()
        _rc(load_library().ils_ws_infer(self._net, N, _ptr(B), _ld(B), _ptr(X0), _ld(X0)),
            "ils_ws_infer")
        return X0

    def save(self, path):
        _rc(load_library().ils_ws_save(self._net, str(path).encode()), "ils_ws_save")

    def load(self, path):
        _rc(load_library().ils_ws_load(self._net, str(path).encode()), "ils_ws_load")

    def get_params(self):
        torch = _torch()
        th = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _rc(load_library().ils_ws_get_params(self._net, _ptr(th)), "ils_ws_get_params")
        return th

    def set_params(self, theta):
        _rc(load_library().ils_ws_set_params(self._net, _ptr(theta.contiguous())), "ils_ws_set_params")

    def forward(self, U):
        """U: (d_in, N) float32 standardised inputs.  Returns Y (n, N) float32."""
        torch = _torch()
        U = U.t().contiguous().t()
        Y = torch.empty((U.shape[1], self.n), dtype=torch.float32, device=U.device).t()
        _rc(load_library().ils_ws_forward(self._net, U.shape[1], _ptr(U), _ptr(Y)), "ils_ws_forward")
        return Y

    def grad(self, U, T):
        torch = _torch()
        U = U.t().contiguous().t()
        T = T.t().contiguous().t()
        g = torch.empty(self.nparams, dtype=torch.float32, device=U.device)
        loss = C.c_double()
        _rc(load_library().ils_ws_grad(self._net, U.shape[1], _ptr(U), _ptr(T), _ptr(g),
                                       C.byref(loss)), "ils_ws_grad")
        return float(loss.value), g

    def adam(self, grad, lr=1e-3):
        _rc(load_library().ils_ws_adam(self._net, _ptr(grad.contiguous()), lr), "ils_ws_adam")


class SparseA:
    """A = [A1; A2] in CSR on the device (ils_csr_*).  rowptr int64 (m + 1),
    colidx int32, val float64 CUDA tensors; they are kept referenced here
    because every solve reads them."""

    def __init__(self, p, q, n, rowptr, colidx, val):
        torch = _torch()
        for t, dt, name in ((rowptr, torch.int64, "rowptr"), (colidx, torch.int32, "colidx"),
                            (val, torch.float64, "val")):
            if not t.is_cuda or t.dtype != dt or t.dim() != 1 or not t.is_contiguous():
                raise ILSError(f"{name} must be a contiguous 1-D {dt} CUDA tensor")
        if rowptr.numel() != p + q + 1 or colidx.numel() != val.numel():
            raise ILSError("CSR arrays have inconsistent sizes")
        self.p, self.q, self.n, self.nnz = p, q, n, val.numel()
        self.m = p + q
        self.device = val.device
        self._keep = (rowptr, colidx, val)
        self._h = handle(self.device)
        A = C.c_void_p()
        _rc(load_library().ils_csr_create(self._h, p, q, n, self.nnz, _ptr(rowptr), _ptr(colidx), _ptr(val),
                                          C.byref(A)), "ils_csr_create")
        self._A = A

    @classmethod
    def from_scipy(cls, S, p, device="cuda"):
        """From a scipy.sparse matrix with m = S.shape[0] rows (A1 = the first p)."""
        torch = _torch()
        S = S.tocsr()
        return cls(p, S.shape[0] - p, S.shape[1],
                   torch.from_numpy(S.indptr.astype("int64")).to(device),
                   torch.from_numpy(S.indices.astype("int32")).to(device),
                   torch.from_numpy(S.data.astype("float64")).to(device))

    def close(self):
        if self._A:
            load_library().ils_csr_destroy(self._A)
            self._A = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _solve(self, fname, b, x0=None, out=None, **kw):
        torch = _torch()
        _check_vec(b, self.m, "b")
        _check_vec(x0, self.n, "x0")
        _check_vec(kw.get("x_ref"), self.n, "x_ref")
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        o = make_opts(**kw)
        info = _Info()
        rc = getattr(load_library(), fname)(self._h, self._A, _ptr(b), _ptr(x0), _ptr(x), C.byref(o),
                                            C.byref(info))
        return x, Info(int(rc), int(info.outer_iters), int(info.inner_iters), float(info.rr),
                       float(info.rel_err), float(info.device_ms))

    def sp_solve(self, b, x0=None, **kw):
        return self._solve("ils_sp_solve_csr", b, x0, **kw)

    def rk_solve(self, b, x0=None, **kw):
        return self._solve("ils_rk_solve_csr", b, x0, **kw)

    def rgs_solve(self, b, x0=None, **kw):
        return self._solve("ils_rgs_solve_csr", b, x0, **kw)

    def gram(self, part):
        torch = _torch()
        G = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        _rc(load_library().ils_csr_gram(self._h, self._A, part, _ptr(G), self.n), "ils_csr_gram")
        return G.t()

    def colpass(self, b):
        torch = _torch()
        g = torch.empty(self.n, dtype=torch.float64, device=self.device)
        c = torch.empty(self.n, dtype=torch.float64, device=self.device)
        rc = load_library().ils_csr_colpass(self._h, self._A, _ptr(b), _ptr(g), _ptr(c))
        return int(rc), g, c

    def residual(self, b, x):
        torch = _torch()
        r = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _rc(load_library().ils_csr_residual(self._h, self._A, _ptr(b), _ptr(x), _ptr(r)), "ils_csr_residual")
        return r

    def csc(self):
        torch = _torch()
        cp = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        ri = torch.empty(self.nnz, dtype=torch.int32, device=self.device)
        cv = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        a1 = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _rc(load_library().ils_csr_export_csc(self._A, _ptr(cp), _ptr(ri), _ptr(cv), _ptr(a1)),
            "ils_csr_export_csc")
        return cp, ri, cv, a1


class _TuneEntry(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("precision", C.c_int32), ("n", C.c_int64), ("K", C.c_int64),
                ("tile", C.c_int32), ("workgroups", C.c_int32), ("ms", C.c_double),
                ("kind", C.c_int32), ("reserved", C.c_int32)]


def tune_gram(A, r0, r1, precision=PREC_FP64, reps=5):
    """Sweep the Gram kernel's launch configurations on rows [r0, r1) of A;
    the fastest becomes the configuration for that shape bucket."""
    e = _TuneEntry()
    _rc(load_library().ils_tune_gram(handle(A.device), r1 - r0, A.shape[1],
                                     C.c_void_p(A.data_ptr() + 8 * r0), _ld(A), precision, reps,
                                     C.byref(e)), "ils_tune_gram")
    return {"kernel": "gram", "precision": int(e.precision), "n": int(e.n), "K": int(e.K),
            "tile": int(e.tile), "workgroups": int(e.workgroups), "ms": float(e.ms), "kind": int(e.kind)}


def _entry(e):
    names = {0: "gram", 1: "batched", 2: "residual"}
    return {"kernel": names[int(e.kernel)], "precision": int(e.precision), "n": int(e.n), "K": int(e.K),
            "tile": int(e.tile), "workgroups": int(e.workgroups), "ms": float(e.ms), "kind": int(e.kind),
            "reserved": int(e.reserved)}


def tune_batched(batch, reps=3, **kw):
    """Sweep the batched solver's launch choices on a Batch (its problems are
    solved by every timed launch); the fastest becomes the choice for that
    bucket."""
    e = _TuneEntry()
    o = make_opts(**kw)
    _rc(load_library().ils_tune_batched(handle(batch.device), len(batch.arr), batch.arr, C.byref(o), reps,
                                        C.byref(e)), "ils_tune_batched")
    return _entry(e)


def tune_residual(A, b, p, x, reps=10):
    """Sweep the residual's launch choices on (A, b, x) (only read)."""
    m, n = A.shape
    e = _TuneEntry()
    _rc(load_library().ils_tune_residual(handle(A.device), p, m - p, n, _ptr(A), _ld(A), _ptr(b), _ptr(x), reps,
                                         C.byref(e)), "ils_tune_residual")
    return _entry(e)


def tune_save(path):
    _rc(load_library().ils_tune_save(str(path).encode()), "ils_tune_save")


def tune_load(path):
    _rc(load_library().ils_tune_load(str(path).encode()), "ils_tune_load")


def tune_clear():
    _rc(load_library().ils_tune_clear(), "ils_tune_clear")
