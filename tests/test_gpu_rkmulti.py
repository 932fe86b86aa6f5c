"""GPU parity of the multi-right-hand-side SP-RK-RGS (ils_rk_solve_multi:
Algorithm 2 for the columns of B sharing A and one index stream) against the
oracle's single-right-hand-side SP-RK-RGS with the same seed, column by
column, through the C ABI: fixed schedules (iterates to 1e-10, ragged last
block, groups of 16 right-hand sides with a ragged last group, both forms),
converged runs with per-column outer and inner stop tests (same outer counts
as the oracle), and the argument errors."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from checks import assert_close

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu


def devA(A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).cuda().t()


def family(p, q, n, r, seed):
    P = W.dense_ils(p, q, n, ratio=0.5, seed=seed, spectral="eig")
    Xs = W.planted_columns(n, r, seed=(seed, r))
    B = np.asfortranarray(P.A @ Xs + 1e-9 * np.random.default_rng(seed).standard_normal((p + q, r)))
    return P, Xs, B


CASES = [(700, 90, 150, 5, 0), (1100, 130, 200, 19, 1), (300, 0, 77, 3, 2), (18000, 2000, 150, 3, 3)]


@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION], ids=["paper", "correction"])
@pytest.mark.parametrize("case", CASES, ids=[f"p{c[0]}_q{c[1]}_n{c[2]}_r{c[3]}" for c in CASES])
def test_fixed_schedule_matches_oracle_per_column(case, form):
    p, q, n, r, seed = case
    P, Xs, B = family(p, q, n, r, seed)
    print(f"[gpu-rkmulti] p={p} q={q} n={n} nrhs={r} form={form}", flush=True)
    inner = 100 if p < 10000 else 70  # ragged: not a multiple of the 32-step block
    X, info, iters = ils.rk_solve_multi(devA(P.A), devA(B), P.p, stop_rule=ils.STOP_FIXED, max_outer=2,
                                        max_inner=inner, seed=7, form=form)
    assert info.status == ils.OK and info.inner_iters == 2 * inner
    assert list(iters) == [2] * r
    Xh = X.cpu().numpy()
    for j in range(r):
        ref, rinfo = O.rk_solve(P.A, B[:, j], P.p, stop_rule=O.STOP_FIXED, max_outer=2, max_inner=inner, seed=7,
                                form=form)
        assert_close(Xh[:, j], ref, 1e-10, what=f"column {j}")


def test_converged_columns_match_oracle():
    """Per-column outer and inner stop tests: each column stops at the
    oracle's outer count (columns retire at different counts: their targets
    differ in size), and lands on the oracle's iterate."""
    p, q, n, r = 500, 100, 50, 6
    P = W.dense_ils(p, q, n, ratio=0.5, seed=11)
    Xs = W.planted_columns(n, r, seed=12)
    Xs[:, 1] *= 1e3  # a column that needs more outer steps to reach tol
    B = np.asfortranarray(P.A @ Xs)
    xr = torch.from_numpy(np.asfortranarray(Xs)).cuda()
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-9, seed=2, form=ils.FORM_CORRECTION, inner_check=50)
    X, info, iters = ils.rk_solve_multi(devA(P.A), devA(B), P.p, x_ref=xr, **kw)
    assert info.status == ils.OK
    Xh = X.cpu().numpy()
    for j in range(r):
        ref, rinfo = O.rk_solve(P.A, B[:, j], P.p, x_ref=Xs[:, j], **kw)
        assert rinfo.status == O.OK
        assert iters[j] == rinfo.outer_iters, (j, iters[j], rinfo.outer_iters)
        assert_close(Xh[:, j], ref, 1e-10, what=f"column {j}")


def test_rr_stop_matches_oracle():
    p, q, n, r = 700, 90, 150, 4
    P, Xs, B = family(p, q, n, r, 5)
    X, info, iters = ils.rk_solve_multi(devA(P.A), devA(B), P.p, tol=1e-10, seed=3, form=ils.FORM_PAPER,
                                        inner_check=150, max_outer=50)
    assert info.status == ils.OK
    Xh = X.cpu().numpy()
    for j in range(r):
        ref, rinfo = O.rk_solve(P.A, B[:, j], P.p, tol=1e-10, seed=3, form=O.FORM_PAPER, inner_check=150,
                                max_outer=50)
        assert iters[j] == rinfo.outer_iters
        assert_close(Xh[:, j], ref, 1e-10, what=f"column {j}")


def test_argument_errors():
    P = W.tiny(0)
    A = devA(P.A)
    B = devA(np.asfortranarray(np.stack([P.b, P.b], axis=1)))
    _, info, _ = ils.rk_solve_multi(A, B, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION)
    assert info.status == ils.ERR_ARG
    _, info, _ = ils.rk_solve_multi(A, B, P.n - 1)  # p < n
    assert info.status == ils.ERR_ARG
