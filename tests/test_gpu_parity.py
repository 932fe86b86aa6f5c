"""GPU parity: the gfx950 library against the FP64 CPU oracle, on the same
seeded inputs, through the C ABI.

Tolerances: 1e-10 relative for the FP64 paths (iterate-for-iterate with the
same schedules and index streams), 1e-6 for the mixed path against x_ILS.
Building blocks are checked at tighter bounds derived from their arithmetic.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from checks import assert_close

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def devA(A):
    """Column-major device copy of a host matrix."""
    return dev(np.asarray(A).T).t()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def banner(msg):
    print(f"[gpu-parity] {msg}", flush=True)


# shapes: tiny (one tile), ragged several-tile, and one with q = 0
SHAPES = [(500, 100, 50), (700, 90, 150), (300, 0, 77), (1100, 130, 200)]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda s: "p%d_q%d_n%d" % s)
def prob(request):
    p, q, n = request.param
    P = W.dense_ils(p, q, n, ratio=0.5, seed=p + q + n)
    banner(f"problem p={p} q={q} n={n}")
    return P, devA(P.A), dev(P.b), dev(P.x_star)


# ----------------------------------------------------------------- building blocks
def test_colpass(prob):
    P, A, b, _ = prob
    rc, g, c = ils.colpass(A, b, P.p)
    assert rc == ils.OK
    assert rel(host(g), O.atjb(P.A, P.b, P.p)) < 1e-13
    A1 = P.A[:P.p]
    assert rel(host(c), (A1 * A1).sum(axis=0)) < 1e-13


def test_gram_f64(prob):
    P, A, b, _ = prob
    for r0, r1 in ((0, P.p), (P.p, P.m), (3, P.p - 5)):
        G = ils.gram(A, r0, r1)
        ref = O.gram(P.A, r0, r1)
        scale = max(np.abs(ref).max(), 1.0)
        assert np.abs(host(G) - ref).max() <= 1e-13 * scale * max(1, r1 - r0) ** 0.5


def test_gram_f32(prob):
    P, A, b, _ = prob
    G = host(ils.gram(A, 0, P.p, precision=ils.PREC_MIXED))
    ref = O.gram(P.A, 0, P.p)
    A1 = P.A[:P.p]
    nrm = np.sqrt((A1 * A1).sum(axis=0))
    # FP32 rounding of the inputs and of a length-p sum: |err| <= ~ (2 + p) u32 |a_i||a_j|
    bound = (2 + P.p) * 2.0 ** -24 * np.outer(nrm, nrm)
    assert np.all(np.abs(G - ref) <= bound)
    assert rel(G, ref) < 1e-5


def test_residual(prob):
    P, A, b, _ = prob
    x = np.random.default_rng(1).standard_normal(P.n)
    r = ils.residual(A, b, P.p, dev(x))
    ref = O.residual(P.A, P.b, P.p, x)
    assert rel(host(r), ref) < 1e-12


@pytest.mark.parametrize("shape", [(1100, 60, 1024), (1200, 90, 1025), (40, 0, 1), (37, 5, 30)],
                         ids=["one_pass_max_n", "two_pass", "n1", "ragged_rows"])
def test_residual_paths(shape):
    """Both residual paths (one pass over A up to n = 1024, two passes above),
    a single column, and fewer 16-row blocks than workgroups with a ragged
    last block."""
    p, q, n = shape
    P = W.dense_ils(p, q, n, ratio=0.5, seed=p + q + n)
    x = np.random.default_rng(2).standard_normal(n)
    r = ils.residual(devA(P.A), dev(P.b), P.p, dev(x))
    ref = O.residual(P.A, P.b, P.p, x)
    assert_close(host(r), ref, 1e-12)


@pytest.mark.parametrize("shape", [(1003, 90, 1000), (45, 3, 70)], ids=["blocks_and_tail", "one_block"])
def test_residual_padded_lda(shape):
    """A view into a taller buffer (lda > m, the rows past m holding NaN):
    the one-pass kernel's rows past m read nothing, so the padding never
    enters r; with a ragged last 16-row block and n not a multiple of 64."""
    p, q, n = shape
    P = W.dense_ils(p, q, n, ratio=0.5, seed=p + q + n + 1)
    m = p + q
    buf = torch.full((n, m + 13), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda()
    A = buf.t()[:m]
    assert A.stride(1) == m + 13
    x = np.random.default_rng(3).standard_normal(n)
    r = ils.residual(A, dev(P.b), P.p, dev(x))
    ref = O.residual(P.A, P.b, P.p, x)
    assert np.all(np.isfinite(host(r)))
    assert_close(host(r), ref, 1e-12)


def test_spd_solve(prob):
    P, A, b, _ = prob
    G1 = O.gram(P.A, 0, P.p)
    R = np.random.default_rng(2).standard_normal((P.n, P.n + 3))
    rc, X = ils.spd_solve(devA(G1), devA(R))
    assert rc == ils.OK
    assert_close(host(X), np.linalg.solve(G1, R), 1e-12)


@pytest.mark.parametrize("n,nrhs", [(1, 1), (63, 2), (64, 64), (65, 1), (128, 129), (129, 64), (192, 3), (300, 301),
                                    (320, 1),
                                    (960, 1), (1000, 1001), (2047, 3), (2048, 2049), (2049, 2),
                                    (2112, 5), (2148, 7), (4096, 3), (4097, 2)])
def test_spd_solve_block_edges(n, nrhs):
    # block edges of the 64-wide Gauss-Jordan: one block, exact multiples, ragged tails
    # (192 and 320: the last pivot block whole, formed ahead of the chain with its
    # row; 300: the ragged block after such steps);
    # up to 32 block rows the elimination is one dataflow launch, above it one
    # launch pair per block step (2048 / 2049, and 2112 / 2148 ending on a
    # full and a ragged block); 4096 and 4097 are the large step-by-step cases
    rng = np.random.default_rng(n)
    if n <= 2048:
        X = rng.standard_normal((3 * n + 5, n))
        G = X.T @ X
    else:  # a nearly square X, shifted to keep G as well conditioned as above
        X = rng.standard_normal((n + 5, n))
        G = X.T @ X + n * np.eye(n)
    R = rng.standard_normal((n, nrhs))
    rc, Y = ils.spd_solve(devA(G), devA(R))
    assert rc == ils.OK
    assert_close(host(Y), np.linalg.solve(G, R), 1e-11)


@pytest.mark.parametrize("n,nrhs", [(1000, 1001), (2048, 65)])
def test_spd_solve_is_reproducible(n, nrhs):
    # the dataflow elimination fixes every tile's update order (one writer per
    # tile and step, steps in order), so repeated calls give the same bits; a
    # tile read before its producer finished, or overwritten while still read,
    # would show as a difference between calls
    rng = np.random.default_rng(n + 3)
    X = rng.standard_normal((2 * n + 9, n))
    G, R = devA(X.T @ X), devA(rng.standard_normal((n, nrhs)))
    rc, Y0 = ils.spd_solve(G, R)
    assert rc == ils.OK
    y0 = host(Y0).copy()
    for _ in range(12):
        rc, Y = ils.spd_solve(G, R)
        assert rc == ils.OK
        assert np.array_equal(host(Y).view(np.uint64), y0.view(np.uint64))


def test_spd_solve_repeated_sizes():
    # the dataflow elimination clears its counters on every call; alternate sizes
    # so that a stale counter or a short scratch buffer would show
    for n, nrhs in ((1000, 1001), (130, 5), (1000, 1001), (700, 2)):
        rng = np.random.default_rng(n + nrhs)
        X = rng.standard_normal((2 * n + 7, n))
        G = X.T @ X
        R = rng.standard_normal((n, nrhs))
        rc, Y = ils.spd_solve(devA(G), devA(R))
        assert rc == ils.OK
        assert_close(host(Y), np.linalg.solve(G, R), 1e-11)


@pytest.mark.parametrize("bad", [0, 63, 64, 100, 129])
def test_spd_solve_detects_indefinite_in_any_block(bad):
    rng = np.random.default_rng(bad + 1)
    Q = np.linalg.qr(rng.standard_normal((130, 130)))[0]
    d = np.linspace(1.0, 2.0, 130)
    d[bad] = -0.5
    G = (Q * d) @ Q.T
    # a permutation that puts the bad direction's weight on a chosen block
    rc, _ = ils.spd_solve(devA(G), devA(np.eye(130)))
    assert rc == ils.ERR_NOT_SPD


def test_spd_solve_detects_indefinite():
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((130, 130)))[0]
    d = np.linspace(1.0, 2.0, 130)
    d[97] = -0.5
    G = (Q * d) @ Q.T
    rc, _ = ils.spd_solve(devA(G), devA(np.eye(130)))
    assert rc == ils.ERR_NOT_SPD


def test_rk_index_stream_is_identical():
    w = np.random.default_rng(4).random(1000) + 1e-3
    for outer in (0, 3):
        j1, j2 = ils.rk_indices(seed=11, outer=outer, t0=5, count=20000, weights=dev(w))
        r1, r2 = O.rk_indices(11, outer, 5, 20000, w)
        assert np.array_equal(host(j1), r1) and np.array_equal(host(j2), r2)


@pytest.mark.parametrize("n,alpha_opt", [(50, 0), (77, 0), (1000, 0), (1000, 10), (4096, 0), (33, 33)])
def test_scd_subsets_are_identical(n, alpha_opt):
    count = 64
    alpha, mask = ils.scd_subsets(seed=7, outer=2, t0=100, count=count, n=n, alpha_opt=alpha_opt)
    alpha, mask = host(alpha), host(mask).view(np.uint32)
    for t in range(count):
        a, mem = O.scd_subset(7, 2, 100 + t, n, alpha_opt)
        assert alpha[t] == a
        bits = np.unpackbits(mask[t].view(np.uint8), bitorder="little")[:n].astype(bool)
        assert np.array_equal(bits, mem)


# ----------------------------------------------------------------- SP (Algorithm 1)
@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_sp_iterates_match_oracle(prob, form):
    P, A, b, _ = prob
    for k in (1, 2, 5):
        x, info = ils.sp_solve(A, b, P.p, stop_rule=ils.STOP_FIXED, max_outer=k, form=form)
        ref, rinfo = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=k, form=form,
                                variant=O.SP_EXPLICIT)
        assert info.status == ils.OK and info.outer_iters == k
        assert_close(host(x), ref, 1e-10)


def test_sp_converged_parity(prob):
    P, A, b, xs = prob
    x, info = ils.sp_solve(A, b, P.p, stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-12)
    ref, rinfo = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-12)
    assert info.status == ils.OK and info.outer_iters == rinfo.outer_iters
    assert_close(host(x), ref, 1e-10)
    assert info.rel_err < 1e-12


def test_sp_rr_stop_matches_oracle(prob):
    P, A, b, _ = prob
    x, info = ils.sp_solve(A, b, P.p, tol=1e-10)
    ref, rinfo = O.sp_solve(P.A, P.b, P.p, tol=1e-10)
    assert info.status == ils.OK and info.outer_iters == rinfo.outer_iters
    # RR (Sec. 5) is a ratio of squared norms: below ~1e-24 (relative residual
    # 1e-12) it is rounding noise of the solve and only its size is comparable
    if rinfo.rr > 1e-24:
        assert info.rr == pytest.approx(rinfo.rr, rel=1e-6)
    else:
        assert info.rr < 1e-24
    assert_close(host(x), ref, 1e-10)


def test_sp_x0_and_resume(prob):
    P, A, b, xs = prob
    x0 = np.random.default_rng(9).standard_normal(P.n)
    x, info = ils.sp_solve(A, b, P.p, x0=dev(x0), stop_rule=ils.STOP_FIXED, max_outer=3)
    ref, _ = O.sp_solve(P.A, P.b, P.p, x0=x0, stop_rule=O.STOP_FIXED, max_outer=3)
    assert_close(host(x), ref, 1e-10)
    # resuming from the returned iterate continues the same sequence
    x2, _ = ils.sp_solve(A, b, P.p, x0=x, stop_rule=ils.STOP_FIXED, max_outer=2)
    ref2, _ = O.sp_solve(P.A, P.b, P.p, x0=x0, stop_rule=O.STOP_FIXED, max_outer=5)
    assert_close(host(x2), ref2, 1e-10)


def test_sp_profiling_modes(prob):
    """Phase events change no result; each mode times what it promises."""
    P, A, b, xs = prob
    kw = dict(stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-10)
    try:
        ils.set_profiling(ils.PROFILE_OFF)
        x0, _ = ils.sp_solve(A, b, P.p, **kw)
        with pytest.raises(ils.ILSError):
            ils.phase_times()
        ils.set_profiling(ils.PROFILE_GRAM)
        x1, _ = ils.sp_solve(A, b, P.p, **kw)
        ph = ils.phase_times()
        assert ph["gram"] > 0.0
        assert all(np.isnan(v) for k, v in ph.items() if k != "gram")
        ils.set_profiling(ils.PROFILE_PHASES)
        x2, _ = ils.sp_solve(A, b, P.p, **kw)
        ph = ils.phase_times()
        assert all(np.isfinite(v) and v >= 0.0 for v in ph.values()) and ph["gram"] > 0.0
        with pytest.raises(ils.ILSError):
            ils.set_profiling(3)
        assert np.array_equal(host(x0), host(x1)) and np.array_equal(host(x0), host(x2))
    finally:
        ils.set_profiling(ils.PROFILE_OFF)


def test_sp_mixed_reaches_x_ils(prob):
    P, A, b, xs = prob
    x, info = ils.sp_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                           stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-8)
    assert info.status == ils.OK
    st, ref = O.normal_solve(P.A, P.b, P.p)
    assert_close(host(x), ref, 1e-6)


def test_sp_error_codes():
    P = W.dense_ils(60, 30, 20, ratio=0.5, seed=3)
    A, b = devA(P.A), dev(P.b)
    x, info = ils.sp_solve(A, b, P.p, max_outer=1, tol=1e-14)
    assert info.status == ils.ERR_NO_CONVERGENCE and info.outer_iters == 1
    Az = P.A.copy()
    Az[:, 4] = 0.0
    out = torch.full((P.n,), 7.0, dtype=torch.float64, device=DEV)
    _, info = ils.sp_solve(devA(Az), b, P.p, out=out)
    assert info.status == ils.ERR_NOT_SPD
    assert torch.all(out == 7.0)  # x untouched
    bn = P.b.copy()
    bn[7] = np.nan
    _, info = ils.sp_solve(A, dev(bn), P.p)
    assert info.status == ils.ERR_NONFINITE
    _, info = ils.sp_solve(devA(P.A[:15]), dev(P.b[:15]), 15)
    assert info.status == ils.ERR_ARG
    _, info = ils.sp_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_PAPER)
    assert info.status == ils.ERR_ARG
    D = W.dense_ils(60, 30, 20, ratio=1.6, seed=3)
    _, info = ils.sp_solve(devA(D.A), dev(D.b), D.p, max_outer=50)
    ref, rinfo = O.sp_solve(D.A, D.b, D.p, max_outer=50)
    assert info.status == rinfo.status


@pytest.mark.parametrize("where", ["b1", "b2", "A1", "A2"])
@pytest.mark.parametrize("val", [np.nan, np.inf])
@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_sp_nonfinite_inputs(where, val, form):
    """A non-finite entry anywhere in A or b gives ERR_NONFINITE and leaves x
    untouched, in both forms (the paper form finds it through the bordered
    Gram products, the correction form through the column pass)."""
    P = W.dense_ils(70, 30, 20, ratio=0.5, seed=4)
    A, b = P.A.copy(), P.b.copy()
    if where == "b1":
        b[5] = val
    elif where == "b2":
        b[P.p + 3] = val
    elif where == "A1":
        A[11, 7] = val
    else:
        A[P.p + 2, 19] = val
    out = torch.full((P.n,), 7.0, dtype=torch.float64, device=DEV)
    _, info = ils.sp_solve(devA(A), dev(b), P.p, out=out, form=form)
    assert info.status == ils.ERR_NONFINITE
    assert torch.all(out == 7.0)


# ----------------------------------------------------------------- SP-RK-RGS (Algorithm 2)
@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_rk_fixed_schedule_matches_oracle(prob, form):
    P, A, b, _ = prob
    x, info = ils.rk_solve(A, b, P.p, stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=700,
                           seed=5, form=form)
    ref, rinfo = O.rk_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=2, max_inner=700,
                            seed=5, form=form)
    assert info.status == ils.OK and info.inner_iters == rinfo.inner_iters == 1400
    assert_close(host(x), ref, 1e-10)


def test_rk_converged_parity():
    P = W.tiny(0)
    A, b, xs = devA(P.A), dev(P.b), dev(P.x_star)
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-9, seed=2, form=ils.FORM_CORRECTION, inner_check=50)
    x, info = ils.rk_solve(A, b, P.p, x_ref=xs, **kw)
    ref, rinfo = O.rk_solve(P.A, P.b, P.p, x_ref=P.x_star, **kw)
    assert info.status == ils.OK and rinfo.status == O.OK
    assert info.outer_iters == rinfo.outer_iters
    assert info.inner_iters == rinfo.inner_iters
    assert_close(host(x), ref, 1e-10)


# ----------------------------------------------------------------- SP-SCD (Algorithm 5)
@pytest.mark.parametrize("alpha,sampling", [(0, ils.SAMPLE_UNIFORM), (1, ils.SAMPLE_NORM),
                                            (7, ils.SAMPLE_UNIFORM), (10 ** 6, ils.SAMPLE_UNIFORM)])
@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_scd_fixed_schedule_matches_oracle(prob, alpha, sampling, form):
    P, A, b, _ = prob
    kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=300, seed=6, alpha=alpha,
              sampling=sampling, form=form)
    x, info = ils.rgs_solve(A, b, P.p, **kw)
    ref, rinfo = O.rgs_solve(P.A, P.b, P.p, **kw)
    assert info.status == ils.OK and info.inner_iters == rinfo.inner_iters == 600
    assert_close(host(x), ref, 1e-10)


@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_scd_converged_parity(form):
    P = W.tiny(0)
    A, b, xs = devA(P.A), dev(P.b), dev(P.x_star)
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-9, seed=4, form=form,
              inner_tol=1e-12 if form == ils.FORM_PAPER else -1.0)
    x, info = ils.rgs_solve(A, b, P.p, x_ref=xs, **kw)
    ref, rinfo = O.rgs_solve(P.A, P.b, P.p, x_ref=P.x_star, **kw)
    assert info.status == ils.OK and rinfo.status == O.OK
    assert info.outer_iters == rinfo.outer_iters
    assert abs(info.inner_iters - rinfo.inner_iters) <= 2 * info.outer_iters
    assert_close(host(x), ref, 1e-10)


def test_scd_mixed_reaches_x_ils():
    P = W.tiny(1)
    A, b, xs = devA(P.A), dev(P.b), dev(P.x_star)
    x, info = ils.rgs_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                            stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-8, seed=1)
    assert info.status == ils.OK
    assert_close(host(x), P.x_star, 1e-6)


@pytest.mark.parametrize("shape", [(500, 100, 50), (700, 90, 150)])
def test_rk_mixed_reaches_x_ils(shape):
    """FP32 inner sweeps (FP32 copy of A1, FP32 w and s) inside FP64
    refinement: the correction form's fixed point is the FP64 x_ILS."""
    P = W.dense_ils(*shape, ratio=0.5, seed=sum(shape))
    A, b, xs = devA(P.A), dev(P.b), dev(P.x_star)
    x, info = ils.rk_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                           stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-8, seed=1)
    assert info.status == ils.OK
    st, x_ils = O.normal_solve(P.A, P.b, P.p)
    assert st == O.OK
    assert_close(host(x), x_ils, 1e-6)
    _, info = ils.rk_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_PAPER)
    assert info.status == ils.ERR_ARG


def test_randomized_error_codes():
    P = W.dense_ils(60, 10, 20, ratio=0.5, seed=3)
    Az = P.A.copy()
    Az[:P.p, 3] = 0.0
    _, info = ils.rk_solve(devA(Az), dev(P.b), P.p)
    assert info.status == ils.ERR_NOT_SPD
    _, info = ils.rgs_solve(devA(Az), dev(P.b), P.p)
    assert info.status == ils.ERR_NOT_SPD
    _, info = ils.rgs_solve(devA(P.A), dev(P.b), P.p, alpha=0, sampling=ils.SAMPLE_NORM)
    assert info.status == ils.ERR_ARG
