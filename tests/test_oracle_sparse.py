"""Pins of the oracle's CSR -> CSC copy and of the sparse input generator.

The CSC copy is pinned against scipy's own conversion (a library routine)
with sorted indices, and on a hand-built matrix with duplicate entries
against the stated order (row, then the value's bit pattern).
"""
import numpy as np
import scipy.sparse as sps

import oracle as O
import workloads as W


def test_csc_matches_scipy():
    for seed, (m, n, dens, p) in enumerate([(50, 7, 0.3, 30), (400, 33, 0.05, 350), (20, 5, 0.9, 0)]):
        S = sps.random(m, n, density=dens, format="csr", random_state=seed)
        cp, ri, cv, a1 = O.csr_to_csc(S, p)
        C = S.tocsc()
        C.sort_indices()
        np.testing.assert_array_equal(cp, C.indptr)
        np.testing.assert_array_equal(ri, C.indices)
        np.testing.assert_array_equal(cv, C.data)
        np.testing.assert_array_equal(a1, [(C.indices[C.indptr[j]:C.indptr[j + 1]] < p).sum()
                                           for j in range(n)])


def test_csc_orders_duplicates_by_value_bits():
    # row 0 holds column 1 twice, row 2 holds column 0 three times
    indptr = np.array([0, 3, 3, 6])
    indices = np.array([1, 0, 1, 0, 0, 0])
    data = np.array([2.0, -1.0, 0.5, 3.0, 1.0, -2.0])
    S = sps.csr_matrix((data, indices, indptr), shape=(3, 2))
    cp, ri, cv, a1 = O.csr_to_csc(S, 1)
    np.testing.assert_array_equal(cp, [0, 4, 6])
    np.testing.assert_array_equal(ri, [0, 2, 2, 2, 0, 0])
    bits = lambda v: np.array(v, dtype=np.float64).view(np.uint64)
    assert list(bits(cv[1:4])) == sorted(bits([3.0, 1.0, -2.0]))
    assert list(bits(cv[4:6])) == sorted(bits([2.0, 0.5]))
    np.testing.assert_array_equal(a1, [1, 2])


def test_sparse_generator_properties():
    P = W.sparse_ils(3000, 300, 120, density=0.05, ratio=0.7, seed=5)
    A = P.A.toarray()
    assert P.A.indices.dtype == np.int32 and P.A.indptr.dtype == np.int64
    A1, A2 = A[:P.p], A[P.p:]
    # the scaled A2 sits just below ratio * sigma_min(A1) (power iteration margin 1e-3)
    r = np.linalg.norm(A2, 2) / np.linalg.svd(A1, compute_uv=False)[-1]
    assert 0.69 < r <= 0.7
    assert np.linalg.eigvalsh(A1.T @ A1 - A2.T @ A2)[0] > 0
    dens = (np.count_nonzero(A1) - P.n) / A1.size
    assert abs(dens - 0.05) < 0.005
    np.testing.assert_allclose(P.A @ P.x_star, P.b, rtol=1e-14, atol=1e-12)
