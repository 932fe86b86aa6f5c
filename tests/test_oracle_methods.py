"""Pins for the oracle's SP, SP-RK-RGS and SP-SCD iterations.

The pins come from the paper's theorems and identities (Thm 2.1, 3.1, 3.2,
4.1; Remark 4.1), closed forms checked with numpy/scipy, and the planted
solution x* of the generated instances.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
import workloads as W


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gnorm(G, v):
    return math.sqrt(float(v @ G @ v))


@pytest.fixture(scope="module")
def prob():
    P = W.tiny(0)
    A, p = P.A, P.p
    G1, G2 = A[:p].T @ A[:p], A[p:].T @ A[p:]
    J = np.diag(np.r_[np.ones(p), -np.ones(P.q)])
    g = A.T @ J @ P.b
    rho = sl.eigh(G2, G1, eigvals_only=True).max()
    return P, G1, G2, g, rho


# ------------------------------------------------------------------ SP
@pytest.mark.parametrize("variant", [O.SP_EXPLICIT, O.SP_CHOLESKY])
@pytest.mark.parametrize("form", [O.FORM_PAPER, O.FORM_CORRECTION])
def test_sp_first_iterate_closed_form(prob, variant, form):
    P, G1, G2, g, rho = prob
    x1, info = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1,
                          variant=variant, form=form)
    assert info.status == O.OK and info.outer_iters == 1
    assert rel(x1, np.linalg.solve(G1, g)) < 1e-13


def test_sp_iterates_match_numpy_recurrence(prob):
    P, G1, G2, g, rho = prob
    x = np.zeros(P.n)
    for k in range(1, 6):
        x = np.linalg.solve(G1, G2 @ x + g)
        for variant in (O.SP_EXPLICIT, O.SP_CHOLESKY):
            xk, _ = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=k,
                               variant=variant)
            assert rel(xk, x) < 1e-13


def test_sp_contracts_in_energy_norm(prob):
    # Thm 2.1: the iteration matrix (A1^T A1)^{-1} A2^T A2 has spectral radius
    # rho < 1 and is self-adjoint in the A1^T A1 inner product, so the error
    # shrinks by at least rho per step in that norm.
    P, G1, G2, g, rho = prob
    assert rho < 1
    errs = []
    for k in range(0, 8):
        xk, _ = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=k,
                           x0=np.ones(P.n))
        errs.append(gnorm(G1, xk - P.x_star))
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 <= rho * e0 * (1 + 1e-9) + 1e-12


def test_sp_outer_count_bound(prob):
    # From x0 = 0: ||e_k|| / ||x*|| <= kappa(A1) rho^k, so the count to tol is
    # at most ceil(ln(tol / kappa) / ln rho).
    P, G1, G2, g, rho = prob
    s = np.linalg.svd(P.A[:P.p], compute_uv=False)
    kappa = s[0] / s[-1]
    for tol in (1e-3, 1e-6, 1e-9):
        bound = math.ceil(math.log(tol / kappa) / math.log(rho))
        x, info = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=tol)
        assert info.status == O.OK
        assert info.outer_iters <= bound
        assert info.rel_err < tol


def test_sp_variants_agree_and_reach_x_ils(prob):
    P, *_ = prob
    xs = []
    for variant in (O.SP_EXPLICIT, O.SP_CHOLESKY):
        for form in (O.FORM_PAPER, O.FORM_CORRECTION):
            x, info = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=30,
                                 variant=variant, form=form)
            xs.append(x)
            assert rel(x, P.x_star) < 1e-12
    for x in xs[1:]:
        assert rel(x, xs[0]) < 1e-12


def test_sp_q_zero_is_exact_in_one_step():
    rng = np.random.default_rng(2)
    A = np.asfortranarray(rng.standard_normal((80, 15)))
    b = rng.standard_normal(80)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    x, info = O.sp_solve(A, b, 80, tol=1e-20)
    assert info.status == O.OK and info.outer_iters == 1
    assert rel(x, ref) < 1e-12


def test_sp_rr_stop_rule(prob):
    P, *_ = prob
    x, info = O.sp_solve(P.A, P.b, P.p, tol=1e-6)
    assert info.status == O.OK and info.rr < 1e-6
    # one iteration fewer would not have met it
    xm, im = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=info.outer_iters - 1)
    assert O.rr(P.A, P.b, P.p, xm) >= 1e-6


def test_sp_error_codes():
    P = W.dense_ils(60, 30, 20, ratio=0.5, seed=3)
    x, info = O.sp_solve(P.A, P.b, P.p, max_outer=1, tol=1e-14)
    assert info.status == O.ERR_NO_CONVERGENCE and info.outer_iters == 1
    A = P.A.copy(order="F")
    A[:, 4] = 0.0                      # A1 loses rank: A^T J A is not SPD
    _, info = O.sp_solve(A, P.b, P.p)
    assert info.status == O.ERR_NOT_SPD
    b = P.b.copy()
    b[7] = np.nan
    _, info = O.sp_solve(P.A, b, P.p)
    assert info.status == O.ERR_NONFINITE
    _, info = O.sp_solve(P.A[:15], P.b[:15], 15)  # p < n
    assert info.status == O.ERR_ARG
    # ratio > 1: A1^T A1 is SPD but the splitting diverges
    D = W.dense_ils(60, 30, 20, ratio=1.6, seed=3)
    _, info = O.sp_solve(D.A, D.b, D.p, max_outer=50)
    assert info.status in (O.ERR_NO_CONVERGENCE, O.ERR_NONFINITE)


# ------------------------------------------------------------------ SP-RK-RGS
def test_rk_inner_fixed_point_is_sp_iterate(prob):
    # Thm 3.1: the RK-RGS inner loop converges to z* = (A1^T A1)^{-1} bhat, the
    # SP iterate; one outer step from x0 = 0 gives (A1^T A1)^{-1} A^T J b.
    P, G1, G2, g, rho = prob
    x1, info = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1,
                          max_inner=40000, seed=3)
    assert rel(x1, np.linalg.solve(G1, g)) < 1e-10


def test_rk_literal_and_incremental_agree(prob):
    P, *_ = prob
    for form in (O.FORM_PAPER, O.FORM_CORRECTION):
        xa, ia = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=2,
                            max_inner=300, seed=5, form=form, variant=O.RK_INCREMENTAL)
        xb, ib = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=2,
                            max_inner=300, seed=5, form=form, variant=O.RK_LITERAL)
        assert rel(xa, xb) < 1e-12


def test_rk_first_step_projection(prob):
    # One RK step from w = 0 projects onto row j1 of A1^T w = bhat, so
    # w = bhat_j1 / ||a_j1||^2 a_j1; one RGS step from z = 0 then sets
    # z_j2 = a_j2^T w / ||a_j2||^2 (Alg. 2 steps 9 and 11).  The indices come
    # from the oracle's own sampler, the arithmetic from numpy.
    P, G1, G2, g, rho = prob
    A1 = P.A[:P.p]
    c = (A1 * A1).sum(axis=0)
    j1, j2 = O.rk_indices(seed=8, outer=0, t0=0, count=1, weights=c)
    a1, a2 = A1[:, j1[0]], A1[:, j2[0]]
    w = g[j1[0]] / c[j1[0]] * a1
    z = np.zeros(P.n)
    z[j2[0]] = a2 @ w / c[j2[0]]
    x1, _ = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1, max_inner=1, seed=8)
    assert rel(x1, z) < 1e-14
    assert abs(a1 @ w - g[j1[0]]) < 1e-12 * abs(g[j1[0]])


@pytest.mark.slow
def test_rk_monte_carlo_rate_bound(prob):
    # Thm 3.2: E||z_t - z*||^2_{G1} <= (1 - s^2/F)^t ||z*||^2_{G1}
    #          + t s_max^2 / F (1 - s^2/F)^t ||w*||^2,  s = sigma_min(A1), F = ||A1||_F^2.
    P, G1, G2, g, rho = prob
    A1 = P.A[:P.p]
    sv = np.linalg.svd(A1, compute_uv=False)
    F = (A1 * A1).sum()
    q = 1 - sv[-1] ** 2 / F
    zs = np.linalg.solve(G1, g)
    ws = A1 @ zs
    for t in (50, 200, 600):
        errs = []
        for seed in range(300):
            z, _ = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1,
                              max_inner=t, seed=1000 + seed)
            errs.append(gnorm(G1, z - zs) ** 2)
        bound = q ** t * gnorm(G1, zs) ** 2 + t * sv[0] ** 2 / F * q ** t * (ws @ ws)
        assert np.mean(errs) <= bound


@pytest.mark.parametrize("form", [O.FORM_PAPER, O.FORM_CORRECTION])
def test_rk_converges_to_x_ils(prob, form):
    P, *_ = prob
    x, info = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-8,
                         form=form, seed=2, max_outer=200,
                         inner_tol=1e-11 if form == O.FORM_PAPER else -1.0)
    assert info.status == O.OK and info.rel_err < 1e-8


def test_rk_zero_column_is_not_spd():
    P = W.dense_ils(60, 10, 20, ratio=0.5, seed=3)
    A = P.A.copy(order="F")
    A[:P.p, 3] = 0.0
    _, info = O.rk_solve(A, P.b, P.p)
    assert info.status == O.ERR_NOT_SPD


# ------------------------------------------------------------------ SP-SCD
def _scd_states(P, t_max, seed, alpha=0, sampling=O.SAMPLE_UNIFORM):
    out = []
    for t in range(t_max + 1):
        beta, _ = O.rgs_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1,
                              max_inner=t, seed=seed, alpha=alpha, sampling=sampling)
        out.append(beta)
    return out


@pytest.mark.parametrize("alpha", [0, 1, 7, 50])
def test_scd_step_properties(prob, alpha):
    # Alg. 5: each step picks j = argmax_{s in tau_t} |r_s| and solves
    # coordinate j exactly (r_{t+1}^{(j)} = 0), and the G1-energy error drops by
    # exactly r_j^2 / G1_jj (the identity in the proof of Thm 4.1).
    P, G1, G2, g, rho = prob
    bstar = np.linalg.solve(G1, g)
    states = _scd_states(P, 25, seed=6, alpha=alpha)
    for t in range(25):
        b0, b1 = states[t], states[t + 1]
        r = g - G1 @ b0
        a, mem = O.scd_subset(seed=6, outer=0, t=t, n=P.n, alpha_opt=alpha)
        cand = np.nonzero(mem)[0]
        j = cand[np.argmax(np.abs(r[cand]))]
        changed = np.nonzero(b1 != b0)[0]
        assert set(changed) <= {j}
        if not len(changed):  # coordinate j was already solved
            assert abs(r[j]) < 1e-10 * np.abs(r).max()
            continue
        assert abs((g - G1 @ b1)[j]) < 1e-10 * np.abs(r).max()
        e0, e1 = gnorm(G1, b0 - bstar) ** 2, gnorm(G1, b1 - bstar) ** 2
        assert e1 == pytest.approx(e0 - r[j] ** 2 / G1[j, j], rel=1e-9, abs=1e-9 * e0)


def test_scd_greedy_is_deterministic_argmax(prob):
    # Remark 4.1, alpha = n: the Motzkin (greedy) choice of the largest residual.
    P, G1, G2, g, rho = prob
    states = _scd_states(P, 15, seed=1, alpha=P.n)
    states2 = _scd_states(P, 15, seed=99, alpha=P.n)
    for t in range(15):
        r = g - G1 @ states[t]
        j = np.nonzero(states[t + 1] != states[t])[0][0]
        assert j == int(np.argmax(np.abs(r)))
        assert np.array_equal(states[t + 1], states2[t + 1])


def test_rcd_mode_frequencies(prob):
    # Remark 4.1, alpha = 1 with norm weights: j drawn with probability
    # G1_jj / trace(G1) -- the RGS/RCD probability.
    P, G1, G2, g, rho = prob
    from scipy import stats
    d = np.diag(G1)
    states = _scd_states(P, 1, seed=0)  # warm the library
    picks = []
    prefix = np.cumsum(d)
    for t in range(20000):
        out = O.philox((t, 0, 0, 0), (7, 0x534344))
        picks.append(O.weighted_index(prefix, O.u01(int(out[1]))))
    counts = np.bincount(picks, minlength=P.n)
    assert stats.chisquare(counts, d / d.sum() * len(picks)).pvalue > 1e-4
    # and the solver follows that stream
    for t in range(5):
        b0, _ = O.rgs_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1, max_inner=t,
                            seed=7, alpha=1, sampling=O.SAMPLE_NORM)
        b1, _ = O.rgs_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1, max_inner=t + 1,
                            seed=7, alpha=1, sampling=O.SAMPLE_NORM)
        changed = np.nonzero(b1 != b0)[0]
        if len(changed):
            assert list(changed) == [picks[t]]
        else:  # the same column twice in a row: its residual is already zero
            assert abs((g - G1 @ b0)[picks[t]]) < 1e-10 * np.abs(g).max()


@pytest.mark.parametrize("form", [O.FORM_PAPER, O.FORM_CORRECTION])
@pytest.mark.parametrize("alpha,sampling", [(0, O.SAMPLE_UNIFORM), (1, O.SAMPLE_NORM),
                                            (50, O.SAMPLE_UNIFORM)])
def test_scd_converges_to_x_ils(prob, form, alpha, sampling):
    P, *_ = prob
    # paper form: the inner solve restarts from 0, so its tolerance bounds the
    # final error; the correction form refines it away
    x, info = O.rgs_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-8,
                          form=form, alpha=alpha, sampling=sampling, seed=4, max_outer=200,
                          inner_tol=1e-11 if form == O.FORM_PAPER else -1.0)
    assert info.status == O.OK and info.rel_err < 1e-8


def test_scd_inner_fixed_point(prob):
    # Thm 4.1: the inner SCD loop converges to beta* = (A1^T A1)^{-1} bhat.
    P, G1, G2, g, rho = prob
    x1, _ = O.rgs_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=1, max_inner=5000,
                        seed=3)
    assert rel(x1, np.linalg.solve(G1, g)) < 1e-12


def test_scd_norm_mode_requires_alpha_one(prob):
    P, *_ = prob
    _, info = O.rgs_solve(P.A, P.b, P.p, alpha=0, sampling=O.SAMPLE_NORM)
    assert info.status == O.ERR_ARG
