"""Python access to the plain FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
baseline leg use this module to check and time the GPU solver; the product
package never imports it.  All arrays are host numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import build as _build

OK, ERR_ARG, ERR_NOT_SPD, ERR_NO_CONVERGENCE, ERR_NONFINITE = 0, -1, -2, -3, -4
STOP_RR, STOP_XREF, STOP_FIXED = 0, 1, 2
FORM_PAPER, FORM_CORRECTION = 0, 1
SP_EXPLICIT, SP_CHOLESKY = 0, 1
RK_INCREMENTAL, RK_LITERAL = 0, 1
SAMPLE_UNIFORM, SAMPLE_NORM = 0, 1


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("stop_rule", C.c_int32), ("form", C.c_int32),
                ("variant", C.c_int32), ("sampling", C.c_int32), ("x_ref", C.c_void_p),
                ("max_outer", C.c_int64), ("max_inner", C.c_int64), ("inner_tol", C.c_double),
                ("inner_check", C.c_int64), ("seed", C.c_uint64), ("stream_offset", C.c_uint64),
                ("alpha", C.c_int64)]


class _Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("pad", C.c_int32), ("outer_iters", C.c_int64),
                ("inner_iters", C.c_int64), ("rr", C.c_double), ("rel_err", C.c_double)]


@dataclasses.dataclass
class Info:
    status: int
    outer_iters: int
    inner_iters: int
    rr: float
    rel_err: float


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or any(
                os.path.getmtime(_build.LIB) < os.path.getmtime(s)
                for s in _build.SRCS + [os.path.join(_build.HERE, "ils_oracle.h")]):
            _build.build()
        L = C.CDLL(_build.LIB)
        P, I64, U64, D = C.c_void_p, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "ora_philox4x64_10": (None, [P, P, P]),
            "ora_mix64": (U64, [U64]),
            "ora_u01": (D, [U64]),
            "ora_uniform_index": (I64, [U64, I64]),
            "ora_weighted_index": (I64, [P, I64, D]),
            "ora_scd_key": (U64, [U64, I64, I64]),
            "ora_rk_indices": (None, [U64, U64, I64, I64, P, I64, P, P]),
            "ora_scd_subset": (None, [U64, U64, I64, I64, I64, P, P]),
            "ora_gram": (None, [I64, I64, I64, P, I64, P]),
            "ora_atjb": (None, [I64, I64, I64, P, I64, P, P]),
            "ora_residual": (None, [I64, I64, I64, P, I64, P, P, P]),
            "ora_set_threads": (None, [C.c_int]),
            "ora_max_threads": (C.c_int, []),
            "ora_rr": (D, [I64, I64, I64, P, I64, P, P]),
            "ora_cholesky": (C.c_int, [I64, P, P]),
            "ora_chol_solve": (None, [I64, P, P, P]),
            "ora_normal_solve": (C.c_int, [I64, I64, I64, P, I64, P, P]),
            "ora_qr_cholesky": (C.c_int, [I64, I64, I64, P, I64, P, P]),
            "ora_opts_default": (None, [P]),
            "ora_mlp_nparams": (I64, [P]),
            "ora_mlp_forward": (None, [P, P, I64, P, P, P, P]),
            "ora_mlp_loss": (D, [P, P, I64, P, P]),
            "ora_mlp_grad": (D, [P, P, I64, P, P, P]),
            "ora_adam_step": (None, [I64, P, P, P, P, I64, D, D, D, D]),
            "ora_bf16_round": (D, [D]),
            "ora_csr_to_csc": (None, [I64, I64, I64, P, P, P, P, P, P, P]),
        }
        for name in ("ora_sp_solve", "ora_rk_solve", "ora_rgs_solve"):
            sig[name] = (C.c_int, [I64, I64, I64, P, I64, P, P, P, P, P])
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f(a):
    """Fortran-ordered float64 view (copy if needed)."""
    return np.asfortranarray(a, dtype=np.float64)


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- PRNG
def philox(ctr, key):
    c = _c(ctr, np.uint64)
    k = _c(key, np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().ora_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def mix64(z: int) -> int:
    return int(lib().ora_mix64(z))


def u01(v: int) -> float:
    return float(lib().ora_u01(v))


def uniform_index(v: int, n: int) -> int:
    return int(lib().ora_uniform_index(v, n))


def weighted_index(prefix, u: float) -> int:
    pr = _c(prefix)
    return int(lib().ora_weighted_index(_ptr(pr), len(pr), u))


def scd_key(K: int, n: int, s: int) -> int:
    return int(lib().ora_scd_key(K, n, s))


def rk_indices(seed, outer, t0, count, weights):
    w = _c(weights)
    j1 = np.zeros(count, dtype=np.int64)
    j2 = np.zeros(count, dtype=np.int64)
    lib().ora_rk_indices(seed, outer, t0, count, _ptr(w), len(w), _ptr(j1), _ptr(j2))
    return j1, j2


def scd_subset(seed, outer, t, n, alpha_opt=0):
    alpha = np.zeros(1, dtype=np.int64)
    member = np.zeros(n, dtype=np.uint8)
    lib().ora_scd_subset(seed, outer, t, n, alpha_opt, _ptr(alpha), _ptr(member))
    return int(alpha[0]), member.astype(bool)


# ---------------------------------------------------------------- dense blocks
def gram(A, r0, r1):
    A = _f(A)
    n = A.shape[1]
    G = np.zeros((n, n), order="F")
    lib().ora_gram(r0, r1, n, _ptr(A), A.shape[0], _ptr(G))
    return G


def atjb(A, b, p):
    A = _f(A)
    m, n = A.shape
    g = np.zeros(n)
    lib().ora_atjb(p, m - p, n, _ptr(A), m, _ptr(_c(b)), _ptr(g))
    return g


def set_threads(t):
    """OpenMP threads of the oracle's parallel loops (results do not depend on it)."""
    lib().ora_set_threads(int(t))


def max_threads():
    return int(lib().ora_max_threads())


def residual(A, b, p, x):
    A = _f(A)
    m, n = A.shape
    r = np.zeros(n)
    lib().ora_residual(p, m - p, n, _ptr(A), m, _ptr(_c(b)), _ptr(_c(x)), _ptr(r))
    return r


def rr(A, b, p, x):
    A = _f(A)
    m, n = A.shape
    return float(lib().ora_rr(p, m - p, n, _ptr(A), m, _ptr(_c(b)), _ptr(_c(x))))


def cholesky(G):
    G = _f(G)
    n = G.shape[0]
    L = np.zeros((n, n), order="F")
    st = lib().ora_cholesky(n, _ptr(G), _ptr(L))
    return st, L


def chol_solve(L, rhs):
    L = _f(L)
    x = np.zeros(L.shape[0])
    lib().ora_chol_solve(L.shape[0], _ptr(L), _ptr(_c(rhs)), _ptr(x))
    return x


def normal_solve(A, b, p):
    A = _f(A)
    m, n = A.shape
    x = np.zeros(n)
    st = lib().ora_normal_solve(p, m - p, n, _ptr(A), m, _ptr(_c(b)), _ptr(x))
    return st, x


def qr_cholesky(A, b, p):
    A = _f(A)
    m, n = A.shape
    x = np.zeros(n)
    st = lib().ora_qr_cholesky(p, m - p, n, _ptr(A), m, _ptr(_c(b)), _ptr(x))
    return st, x


# ---------------------------------------------------------------- solvers
def _solve(fname, A, b, p, x0=None, tol=1e-6, stop_rule=STOP_RR, form=FORM_PAPER,
           variant=0, sampling=SAMPLE_UNIFORM, x_ref=None, max_outer=20000,
           max_inner=-1, inner_tol=-1.0, inner_check=-1, seed=0, stream_offset=0,
           alpha=0, lda=None):
    A = _f(A)
    m, n = A.shape
    b = _c(b)
    x0a = None if x0 is None else _c(x0)
    xr = None if x_ref is None else _c(x_ref)
    o = _Opts()
    lib().ora_opts_default(C.byref(o))
    o.tol, o.stop_rule, o.form, o.variant, o.sampling = tol, stop_rule, form, variant, sampling
    o.x_ref = _ptr(xr)
    o.max_outer, o.max_inner, o.inner_tol, o.inner_check = max_outer, max_inner, inner_tol, inner_check
    o.seed, o.stream_offset, o.alpha = seed, stream_offset, alpha
    x = np.full(n, np.nan)
    info = _Info()
    st = getattr(lib(), fname)(p, m - p, n, _ptr(A), m if lda is None else lda, _ptr(b),
                               _ptr(x0a), _ptr(x), C.byref(o), C.byref(info))
    return x, Info(int(st), int(info.outer_iters), int(info.inner_iters), float(info.rr),
                   float(info.rel_err))


def sp_solve(A, b, p, **kw):
    """SP (Algorithm 1).  variant=SP_EXPLICIT (B = G1^-1 G2 and c = G1^-1 A^T J b
    of the update (Sec23) formed once) or SP_CHOLESKY (triangular solves)."""
    return _solve("ora_sp_solve", A, b, p, **kw)


def rk_solve(A, b, p, **kw):
    """SP-RK-RGS (Algorithm 2).  variant=RK_INCREMENTAL or RK_LITERAL."""
    return _solve("ora_rk_solve", A, b, p, **kw)


def rgs_solve(A, b, p, **kw):
    """SP-SCD (Algorithm 5); alpha=1 with sampling=SAMPLE_NORM is SP-RCD."""
    return _solve("ora_rgs_solve", A, b, p, **kw)


# ---------------------------------------------------------------- warm-start MLP
def _dims(d):
    return np.asarray(d, dtype=np.int64)


def mlp_nparams(d):
    dd = _dims(d)
    return int(lib().ora_mlp_nparams(_ptr(dd)))


def mlp_forward(d, theta, U):
    """U: (d0, B) array, one sample per column.  Returns Y (d3, B), H1, H2."""
    dd = _dims(d)
    th = _c(theta)
    Uf = _f(U)
    B = Uf.shape[1]
    Y = np.zeros((d[3], B), order="F")
    H1 = np.zeros((d[1], B), order="F")
    H2 = np.zeros((d[2], B), order="F")
    lib().ora_mlp_forward(_ptr(dd), _ptr(th), B, _ptr(Uf), _ptr(Y), _ptr(H1), _ptr(H2))
    return Y, H1, H2


def mlp_loss(d, theta, U, T):
    dd = _dims(d)
    Uf, Tf = _f(U), _f(T)
    return float(lib().ora_mlp_loss(_ptr(dd), _ptr(_c(theta)), Uf.shape[1], _ptr(Uf), _ptr(Tf)))


def mlp_grad(d, theta, U, T):
    """Returns (loss, gradient of the loss with respect to theta)."""
    dd = _dims(d)
    th = _c(theta)
    Uf, Tf = _f(U), _f(T)
    g = np.zeros_like(th)
    loss = lib().ora_mlp_grad(_ptr(dd), _ptr(th), Uf.shape[1], _ptr(Uf), _ptr(Tf), _ptr(g))
    return float(loss), g


def adam_step(w, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays w, m, v with gradient g at step t >= 1."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gc = _c(g)
    lib().ora_adam_step(len(w), _ptr(w), _ptr(m), _ptr(v), _ptr(gc), t, lr, beta1, beta2, eps)


def bf16_round(a):
    """Round every entry to the nearest bfloat16 value (ties to even)."""
    f = np.vectorize(lambda x: lib().ora_bf16_round(float(x)), otypes=[np.float64])
    return f(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- sparse
def csr_to_csc(S, p):
    """(colptr, rowidx, val, a1len) of the CSC copy of scipy CSR matrix S:
    rows ascending per column, duplicates by value bits; a1len = rows < p."""
    S = S.tocsr()
    m, n = S.shape
    rp = np.ascontiguousarray(S.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(S.indices, dtype=np.int32)
    v = np.ascontiguousarray(S.data, dtype=np.float64)
    cp = np.zeros(n + 1, dtype=np.int64)
    ri = np.zeros(len(v), dtype=np.int32)
    cv = np.zeros(len(v), dtype=np.float64)
    a1 = np.zeros(n, dtype=np.int32)
    lib().ora_csr_to_csc(m, n, p, _ptr(rp), _ptr(ci), _ptr(v), _ptr(cp), _ptr(ri), _ptr(cv), _ptr(a1))
    return cp, ri, cv, a1
