"""GPU parity of the sparse (CSR) path against the oracle.

The CSC copy must equal the oracle's bit for bit.  The building blocks and
the three methods are compared with the dense FP64 oracle on the densified
matrix (the same mathematical objects): Gram products, A^T J b and the
residual to 1e-13 relative, SP iterates to 1e-10 (FIXED schedules), SP-RK-
RGS and SP-SCD iterate for iterate with the same seeds to 1e-10.
"""
import numpy as np
import pytest
import scipy.sparse as sps

import oracle as O
import workloads as W
from checks import assert_close

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def banner(msg):
    print(f"[gpu-sparse] {msg}", flush=True)


# (p, q, n, density): ragged, q = 0, columns longer than the in-LDS sort (4096 + )
CASES = [(3000, 300, 120, 0.05), (2000, 0, 90, 0.06), (9000, 900, 24, 0.5)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "p%d_q%d_n%d" % c[:3])
def sp(request):
    p, q, n, d = request.param
    banner(f"sparse p={p} q={q} n={n} density={d}")
    P = W.sparse_ils(p, q, n, density=d, ratio=0.7, seed=p + n)
    S = ils.SparseA.from_scipy(P.A, p)
    yield P, P.A.toarray(order="F"), S, dev(P.b), dev(P.x_star)
    S.close()


def test_csc_copy_is_exact(sp):
    P, _, S, _, _ = sp
    cp, ri, cv, a1 = (host(t) for t in S.csc())
    ocp, ori, ocv, oa1 = O.csr_to_csc(P.A, P.p)
    np.testing.assert_array_equal(cp, ocp)
    np.testing.assert_array_equal(ri, ori)
    np.testing.assert_array_equal(cv.view(np.uint64), ocv.view(np.uint64))
    np.testing.assert_array_equal(a1, oa1)


def test_colpass_and_residual(sp):
    P, A, S, b, _ = sp
    rc, g, c = S.colpass(b)
    assert rc == ils.OK
    assert rel(host(g), O.atjb(A, P.b, P.p)) < 1e-13
    assert rel(host(c), np.diag(O.gram(A, 0, P.p))) < 1e-13
    x = np.random.default_rng(1).standard_normal(P.n)
    r = S.residual(b, dev(x))
    ref = O.residual(A, P.b, P.p, x)
    assert np.linalg.norm(host(r) - ref) <= 1e-12 * np.linalg.norm(O.atjb(A, P.b, P.p))


def test_gram_parts(sp):
    P, A, S, _, _ = sp
    for part, (r0, r1) in enumerate([(0, P.p), (P.p, P.m)]):
        G = host(S.gram(part))
        ref = O.gram(A, r0, r1)
        if r1 == r0:
            assert np.all(G == 0.0)
            continue
        assert np.linalg.norm(G - ref) <= 1e-13 * np.linalg.norm(ref)
        np.testing.assert_array_equal(G, G.T)
        for _ in range(3):  # run to run, bit for bit
            np.testing.assert_array_equal(host(S.gram(part)).view(np.uint64), G.view(np.uint64))


@pytest.mark.parametrize("form", ["paper", "correction"])
def test_sp_fixed_schedule(sp, form):
    P, A, S, b, _ = sp
    f = ils.FORM_PAPER if form == "paper" else ils.FORM_CORRECTION
    x0 = np.random.default_rng(2).standard_normal(P.n)
    for k in (1, 5):
        x, inf = S.sp_solve(b, x0=dev(x0), stop_rule=ils.STOP_FIXED, max_outer=k, form=f)
        assert inf.status == ils.OK and inf.outer_iters == k
        ref, _ = O.sp_solve(A, P.b, P.p, x0=x0, stop_rule=O.STOP_FIXED, max_outer=k,
                            variant=O.SP_EXPLICIT, form=f)
        assert_close(host(x), ref, 1e-10)


def test_sp_converges_to_planted(sp):
    P, A, S, b, xs = sp
    x, inf = S.sp_solve(b, stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-9)
    assert inf.status == ils.OK
    ref, rinf = O.sp_solve(A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-9,
                           variant=O.SP_EXPLICIT)
    assert inf.outer_iters == rinf.outer_iters
    assert_close(host(x), ref, 1e-10)
    # the stop rule itself is normwise: ||x - x*|| / ||x*|| < 1e-9
    assert rel(host(x), P.x_star) < 1e-9
    x, inf = S.sp_solve(b, stop_rule=ils.STOP_RR, tol=1e-16)
    assert inf.status == ils.OK and inf.rr < 1e-16


@pytest.mark.parametrize("form", ["paper", "correction"])
def test_rk_fixed_schedule(sp, form):
    P, A, S, b, _ = sp
    f = ils.FORM_PAPER if form == "paper" else ils.FORM_CORRECTION
    kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=300, seed=7, form=f)
    x, inf = S.rk_solve(b, **kw)
    assert inf.status == ils.OK
    ref, _ = O.rk_solve(A, P.b, P.p, **kw)
    assert_close(host(x), ref, 1e-10)


def test_rk_mixed_column_lengths():
    # A1 columns above and below the sparse inner step's register capacity
    # (2048 entries) in one schedule: the step alternates between its register
    # form and its loop form and loads the next step's columns in either
    p, q, n = 5000, 500, 40
    banner(f"sparse RK-RGS, mixed column lengths p={p} q={q} n={n}")
    P = W.sparse_ils(p, q, n, density=0.05, ratio=0.7, seed=11)
    A = P.A.toarray(order="F")
    rng = np.random.default_rng(5)
    for c in (3, 17, 18, 30):
        A[:p, c] += rng.standard_normal(p)
    S = ils.SparseA.from_scipy(sps.csr_matrix(A), p)
    try:
        b = dev(P.b)
        for f in (ils.FORM_PAPER, ils.FORM_CORRECTION):
            kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=300, seed=7, form=f)
            x, inf = S.rk_solve(b, **kw)
            assert inf.status == ils.OK
            ref, _ = O.rk_solve(A, P.b, P.p, **kw)
            assert_close(host(x), ref, 1e-10)
    finally:
        S.close()


@pytest.mark.parametrize("alpha", [0, 1])
def test_scd_fixed_schedule(sp, alpha):
    P, A, S, b, _ = sp
    kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=200, seed=9, alpha=alpha,
              sampling=ils.SAMPLE_NORM if alpha == 1 else ils.SAMPLE_UNIFORM)
    x, inf = S.rgs_solve(b, **kw)
    assert inf.status == ils.OK
    ref, _ = O.rgs_solve(A, P.b, P.p, **kw)
    assert_close(host(x), ref, 1e-10)


def test_randomized_converge(sp):
    P, A, S, b, xs = sp
    x, inf = S.rgs_solve(b, stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6,
                         form=ils.FORM_CORRECTION, seed=3)
    assert inf.status == ils.OK and inf.rel_err < 1e-6
    if P.n <= 120:
        x, inf = S.rk_solve(b, stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6,
                            form=ils.FORM_CORRECTION, seed=3)
        assert inf.status == ils.OK and inf.rel_err < 1e-6


def test_errors():
    rp = dev(np.array([0, 1, 3], dtype=np.int64))
    ci = dev(np.array([0, 1, 5], dtype=np.int32))     # column 5 out of range for n = 2
    v = dev(np.array([1.0, 2.0, 3.0]))
    with pytest.raises(ils.ILSError):
        ils.SparseA(1, 1, 2, rp, ci, v)
    ci_ok = dev(np.array([0, 1, 0], dtype=np.int32))
    with pytest.raises(ils.ILSError):
        ils.SparseA(1, 1, 2, rp, ci_ok, dev(np.array([1.0, np.nan, 3.0])))
    with pytest.raises(ils.ILSError):                 # rowptr[m] != nnz
        ils.SparseA(1, 1, 2, dev(np.array([0, 1, 2], dtype=np.int64)), ci_ok, v)
    P = W.sparse_ils(300, 30, 20, density=0.2, seed=1)
    S = ils.SparseA.from_scipy(P.A, P.p)
    _, inf = S.sp_solve(dev(P.b), form=ils.FORM_CORRECTION, precision=ils.PREC_MIXED)
    assert inf.status == ils.ERR_ARG
    bad = P.b.copy()
    bad[3] = np.inf
    _, inf = S.sp_solve(dev(bad))
    assert inf.status == ils.ERR_NONFINITE
    # rank-deficient A1 (column 19 of A1 is zero): A1^T A1 is singular, not SPD
    Q = sps.csr_matrix(np.vstack([np.eye(20)[:19], np.eye(20)[:1], np.ones((4, 20))]))
    S2 = ils.SparseA.from_scipy(Q, 20)
    _, inf = S2.sp_solve(dev(np.ones(24)))
    assert inf.status == ils.ERR_NOT_SPD
    S2.close()
    S.close()
