"""Seeded synthetic inputs for the indefinite least squares (ILS) solvers.

This module only builds inputs: matrices, right-hand sides, planted solutions.
It holds none of the solvers' arithmetic and is shared by the CPU oracle's
tests, the GPU parity tests and the benchmark.

The dense family follows the problem statement of Sec. 1 (A = [A1; A2],
J = diag(I_p, -I_q)): A1 and A2 get i.i.d. N(0,1) entries, A2 is then
rescaled so that ||A2||_2 = ratio * sigma_min(A1).  With ratio < 1 this keeps
A^T J A symmetric positive definite, the standing assumption (Sec12)-(Sec13).
A planted x* gives b = A x* (+ optional noise), so x_ILS = x* when there is no
noise.  Arrays come out column-major (Fortran order), float64.

The paper's own experiment family (Sec. 5.2 / 5.3: A1 = U[0,1), A2 = 7 * eye)
is available as `paper_family`.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class DenseILS:
    A: np.ndarray          # (m, n) float64, Fortran order
    b: np.ndarray          # (m,)
    p: int
    q: int
    x_star: np.ndarray     # planted solution (n,), or None
    ratio: float           # ||A2||_2 / sigma_min(A1) after scaling
    seed: object

    @property
    def m(self) -> int:
        return self.p + self.q

    @property
    def n(self) -> int:
        return self.A.shape[1]


def _rng(seed):
    if isinstance(seed, (tuple, list)):
        return np.random.default_rng(list(seed))
    return np.random.default_rng(seed)


def dense_ils(p: int, q: int, n: int, ratio: float = 0.5, seed=0,
              noise: float = 0.0, a1: np.ndarray | None = None,
              spectral: str = "svd") -> DenseILS:
    """Gaussian ILS instance with A2 scaled to ||A2||_2 = ratio * sigma_min(A1).

    Draw order from numpy.random.default_rng(seed): A1 (p x n), A2 (q x n),
    x* (n), noise (m).  `a1` lets two instances share the same A1 (the
    ratio-0.5 and ratio-0.9 variants of one problem).  spectral="svd" takes
    sigma_min(A1) and ||A2||_2 from singular values; "eig" from the extreme
    eigenvalues of A1^T A1 and A2^T A2 (cheaper, for large batches).
    """
    rng = _rng(seed)
    A1 = rng.standard_normal((p, n)) if a1 is None else np.array(a1, dtype=np.float64)
    if a1 is not None:
        rng.standard_normal((p, n))  # keep the stream position identical
    A2 = rng.standard_normal((q, n))
    x_star = rng.standard_normal(n)
    e = rng.standard_normal(p + q)
    if q > 0:
        if spectral == "eig":
            smin = float(np.sqrt(np.linalg.eigvalsh(A1.T @ A1)[0]))
            a2n = float(np.sqrt(np.linalg.eigvalsh(A2.T @ A2)[-1]))
        else:
            smin = np.linalg.svd(A1, compute_uv=False)[-1]
            a2n = np.linalg.svd(A2, compute_uv=False)[0]
        A2 = A2 * (ratio * smin / a2n)
    A = np.asfortranarray(np.vstack([A1, A2]))
    b = A @ x_star
    if noise:
        b = b + noise * e
    return DenseILS(A=A, b=np.ascontiguousarray(b), p=p, q=q, x_star=x_star,
                    ratio=ratio, seed=seed)


def tiny(seed=0) -> DenseILS:
    """A1 500x50, A2 100x50, ratio 0.5, b = A x*, no noise."""
    return dense_ils(500, 100, 50, ratio=0.5, seed=seed)


def large(ratio: float = 0.5, seed=1) -> DenseILS:
    """A1 18000x1000, A2 2000x1000, b = A x* + 1e-8 N(0,1).

    The ratio-0.5 and ratio-0.9 variants use the same seed and hence share
    A1, A2 (before scaling) and x*.
    """
    return dense_ils(18000, 2000, 1000, ratio=ratio, seed=seed, noise=1e-8)


def batched_sizes(count: int = 4096, seed: int = 3, lo: int = 32, hi: int = 256):
    """Per-instance n ~ U{lo..hi}, p = 4n, q = floor(n/2)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(lo, hi + 1, size=count)
    return [(4 * int(n), int(n) // 2, int(n)) for n in ns]


def batched_instance(i: int, n: int, seed: int = 3) -> DenseILS:
    p, q = 4 * n, n // 2
    return dense_ils(p, q, n, ratio=0.5, seed=(seed, i), spectral="eig")


def batched(count: int = 4096, seed: int = 3, threads: int = 16):
    """The batch: instance i has n_i from batched_sizes and seed (seed, i)."""
    import concurrent.futures as cf

    from threadpoolctl import threadpool_limits
    sizes = batched_sizes(count, seed)
    with threadpool_limits(1), cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda a: batched_instance(a[0], a[1][2], seed), enumerate(sizes)))


def planted_columns(n: int, nrhs: int, seed, basis=None, noise: float = 0.0) -> np.ndarray:
    """Planted solutions X* (n x nrhs, Fortran order) for right-hand sides
    B = A X* that share A: i.i.d. N(0,1) entries, or, given an orthonormal
    basis U (n x r), X* = U theta + noise * eps with theta ~ N(0, I_r) and
    eps ~ N(0, I_n) per column (draw order theta, eps)."""
    rng = _rng(seed)
    if basis is None:
        return np.asfortranarray(rng.standard_normal((nrhs, n)).T)
    theta = rng.standard_normal((nrhs, basis.shape[1])).T
    eps = rng.standard_normal((nrhs, n)).T
    return np.asfortranarray(basis @ theta + noise * eps)


# Warm-start family: one A of the 18000 + 2000 x 1000 shape (ratio 0.5),
# solutions in a random 32-dimensional subspace plus 1e-3 noise, and the
# network input = every 10th row of b (2000 rows).
WS_RANK = 32
WS_NOISE = 1e-3
WS_IN_STRIDE = 10


def ws_problem(seed: int = 4):
    """(A's instance, U): A as `large` with ratio 0.5 from `seed` (no noise),
    U the Q factor of a 1000 x 32 Gaussian matrix drawn from (seed, 1)."""
    P = dense_ils(18000, 2000, 1000, ratio=0.5, seed=seed)
    U, _ = np.linalg.qr(_rng((seed, 1)).standard_normal((P.n, WS_RANK)))
    return P, np.asfortranarray(U)


def ws_in_rows(m: int) -> np.ndarray:
    return np.arange(0, m, WS_IN_STRIDE, dtype=np.int64)


def ws_solutions(U: np.ndarray, count: int, seed) -> np.ndarray:
    """count planted x = U theta + 1e-3 eps (n x count)."""
    return planted_columns(U.shape[0], count, seed, basis=U, noise=WS_NOISE)


@dataclasses.dataclass
class SparseILS:
    A: object              # scipy.sparse.csr_matrix (m, n), float64, int32 indices
    b: np.ndarray
    p: int
    q: int
    x_star: np.ndarray
    ratio: float
    seed: object

    @property
    def m(self) -> int:
        return self.p + self.q

    @property
    def n(self) -> int:
        return self.A.shape[1]


def sparse_ils(p: int, q: int, n: int, density: float = 0.005, ratio: float = 0.7, seed=2,
               power_iters: int = 200) -> SparseILS:
    """Sparse ILS instance: every entry of A (m x n) is nonzero independently
    with probability `density` (a Bernoulli process over the row-major
    positions, drawn as geometric gaps) with an N(0,1) value; A1[i, i] += 1
    for i < n (full rank); A2 scaled to ||A2||_2 = ratio * sigma_min(A1),
    with ||A2||_2 from `power_iters` power iterations on A2^T A2 times
    (1 + 1e-3) and sigma_min(A1) from the eigenvalues of the dense A1^T A1.
    x* ~ N(0, I), b = A x*.  Draw order: gaps, values, power-iteration start,
    x*."""
    import scipy.sparse as sps
    rng = _rng(seed)
    m = p + q
    total = m * n
    pos = np.empty(0, dtype=np.int64)
    last = -1
    while True:
        want = int((total - last) * density * 1.05) + 1024
        gaps = rng.geometric(density, size=want).astype(np.int64)
        chunk = last + np.cumsum(gaps)
        pos = np.concatenate([pos, chunk[chunk < total]])
        if chunk[-1] >= total:
            break
        last = int(chunk[-1])
    vals = rng.standard_normal(len(pos))
    rows, cols = pos // n, pos % n
    d = np.arange(min(n, p))
    A = sps.coo_matrix((np.concatenate([vals, np.ones(len(d))]),
                        (np.concatenate([rows, d]), np.concatenate([cols, d]))), shape=(m, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    v = rng.standard_normal(n)
    x_star = rng.standard_normal(n)
    A1, A2 = A[:p], A[p:]
    if q > 0:
        v /= np.linalg.norm(v)
        lam = 0.0
        for _ in range(power_iters):
            u = A2.T @ (A2 @ v)
            lam = float(np.linalg.norm(u))
            v = u / lam
        a2n = np.sqrt(lam) * (1 + 1e-3)
        smin = float(np.sqrt(np.linalg.eigvalsh((A1.T @ A1).toarray())[0]))
        A2 = A2 * (ratio * smin / a2n)
        A = sps.vstack([A1, A2]).tocsr()
        A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int64)
    b = A @ x_star
    return SparseILS(A=A, b=np.ascontiguousarray(b), p=p, q=q, x_star=x_star, ratio=ratio, seed=seed)


def sparse_large(seed: int = 2) -> SparseILS:
    """p = 180000, q = 20000, n = 4000, density 0.005, ratio 0.7."""
    return sparse_ils(180000, 20000, 4000, density=0.005, ratio=0.7, seed=seed)


def paper_family(p: int, q: int, n: int, seed=0) -> DenseILS:
    """The experiment family of Sec. 5.2 (q = n) and Sec. 5.3 (q = 1).

    A1 = U[0,1) p x n, A2 = 7 * (first q rows of I_n), b1, b2 = U[0,1).
    There is no planted solution (x_star is None).
    """
    rng = _rng(seed)
    A1 = rng.random((p, n))
    A2 = np.zeros((q, n))
    k = min(q, n)
    A2[np.arange(k), np.arange(k)] = 7.0
    b = rng.random(p + q)
    A = np.asfortranarray(np.vstack([A1, A2]))
    return DenseILS(A=A, b=b, p=p, q=q, x_star=None, ratio=float("nan"), seed=seed)
