"""Pins for the oracle's direct solutions and dense building blocks.

Every check compares the oracle with something other than itself: the planted
solution, numpy/scipy library routines used as textbook references, or an
identity the paper states (Sec. 1, Sec. 2).
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import workloads as W


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_gram_and_atjb_match_numpy(tiny):
    A, b, p = tiny.A, tiny.b, tiny.p
    G1 = O.gram(A, 0, p)
    G2 = O.gram(A, p, tiny.m)
    assert rel(G1, A[:p].T @ A[:p]) < 1e-14
    assert rel(G2, A[p:].T @ A[p:]) < 1e-14
    # A^T J A = A1^T A1 - A2^T A2 (Sec. 2)
    J = np.diag(np.r_[np.ones(p), -np.ones(tiny.q)])
    assert rel(G1 - G2, A.T @ J @ A) < 1e-13
    assert rel(O.atjb(A, b, p), A.T @ J @ b) < 1e-14


def test_residual_and_rr_definition(tiny):
    A, b, p = tiny.A, tiny.b, tiny.p
    J = np.diag(np.r_[np.ones(p), -np.ones(tiny.q)])
    x = np.random.default_rng(5).standard_normal(tiny.n)
    r = O.residual(A, b, p, x)
    assert rel(r, A.T @ J @ (b - A @ x)) < 1e-13
    # RR at x0 = 0 is exactly 1 and vanishes at the planted solution (Sec. 5)
    assert O.rr(A, b, p, np.zeros(tiny.n)) == pytest.approx(1.0, abs=1e-15)
    assert O.rr(A, b, p, tiny.x_star) < 1e-26


def test_normal_solve_recovers_planted_solution(tiny):
    st, x = O.normal_solve(tiny.A, tiny.b, tiny.p)
    assert st == O.OK
    assert rel(x, tiny.x_star) < 1e-12


def test_normal_solve_matches_numpy_solve():
    rng = np.random.default_rng(11)
    P = W.dense_ils(120, 30, 40, ratio=0.8, seed=11)
    # a right-hand side with no planted solution
    b = rng.standard_normal(P.m)
    J = np.diag(np.r_[np.ones(P.p), -np.ones(P.q)])
    ref = np.linalg.solve(P.A.T @ J @ P.A, P.A.T @ J @ b)
    st, x = O.normal_solve(P.A, b, P.p)
    assert st == O.OK and rel(x, ref) < 1e-12
    # residual orthogonality A^T J (b - A x_ILS) = 0 (Sec12)
    assert np.linalg.norm(O.residual(P.A, b, P.p, x)) < 1e-10 * np.linalg.norm(P.A.T @ J @ b)


def test_qr_cholesky_agrees_with_normal_equation():
    rng = np.random.default_rng(12)
    P = W.dense_ils(90, 20, 25, ratio=0.6, seed=12)
    b = rng.standard_normal(P.m)
    st1, x1 = O.normal_solve(P.A, b, P.p)
    st2, x2 = O.qr_cholesky(P.A, b, P.p)
    assert st1 == st2 == O.OK
    assert rel(x2, x1) < 1e-11


def test_q_zero_is_ordinary_least_squares():
    rng = np.random.default_rng(13)
    A = np.asfortranarray(rng.standard_normal((70, 12)))
    b = rng.standard_normal(70)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    for f in (O.normal_solve, O.qr_cholesky):
        st, x = f(A, b, 70)
        assert st == O.OK and rel(x, ref) < 1e-12


def test_not_spd_is_reported():
    # A2 scaled past sigma_min(A1): A^T J A is indefinite (Sec13 fails)
    P = W.dense_ils(60, 30, 20, ratio=1.5, seed=3)
    J = np.diag(np.r_[np.ones(P.p), -np.ones(P.q)])
    assert np.linalg.eigvalsh(P.A.T @ J @ P.A).min() < 0
    st, _ = O.normal_solve(P.A, P.b, P.p)
    assert st == O.ERR_NOT_SPD
    st, _ = O.qr_cholesky(P.A, P.b, P.p)
    assert st == O.ERR_NOT_SPD


def test_cholesky_matches_numpy():
    G = O.gram(W.tiny(1).A, 0, 500)
    st, L = O.cholesky(G)
    assert st == O.OK
    assert rel(L, np.linalg.cholesky(G)) < 1e-13
    rhs = np.arange(G.shape[0], dtype=float)
    assert rel(O.chol_solve(L, rhs), np.linalg.solve(G, rhs)) < 1e-12


def test_spd_invariant_of_generated_instances(tiny):
    # A1^T A1 SPD, and the generalized eigenvalues of (A2^T A2, A1^T A1) lie in
    # [0, ratio^2] -- the spectral fact behind Theorem 2.1.
    A, p = tiny.A, tiny.p
    G1, G2 = A[:p].T @ A[:p], A[p:].T @ A[p:]
    lam = sl.eigh(G2, G1, eigvals_only=True)
    assert lam.min() > -1e-12
    assert lam.max() <= tiny.ratio ** 2 * (1 + 1e-10)
    assert np.linalg.eigvalsh(G1 - G2).min() > 0


def test_thread_count_does_not_change_results():
    """The oracle's parallel loops write disjoint entries with sums in index
    order, so its results are the same bits for any OpenMP thread count."""
    import oracle as O
    import workloads as W
    P = W.dense_ils(700, 90, 150, seed=21)
    outs = []
    try:
        for t in (1, 3, 8):
            O.set_threads(t)
            x, info = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=4, variant=O.SP_CHOLESKY)
            outs.append((x, O.gram(P.A, 0, P.p)))
    finally:
        O.set_threads(max(1, len(__import__("os").sched_getaffinity(0))))
    for x, G in outs[1:]:
        assert np.array_equal(x, outs[0][0]) and np.array_equal(G, outs[0][1])
