"""GPU parity on the launch shapes that only large problems reach.

* SP-RK-RGS (Algorithm 2) runs its inner steps in blocks of 32 over row
  slices of A1 whose height grows with p: 16 rows up to p = 4096, 80 rows at
  p = 18000 (the headline problem's A1), and more than the 128 rows one LDS
  chunk holds above p = 32768.  Fixed schedules (several whole blocks and a
  ragged last one) are compared with the oracle at 1e-10 in FP64, and the
  mixed form's converged result with x_ILS at 1e-6.
* SP-SCD (Algorithm 5) keeps its residual in LDS up to n = 4096 and in global
  memory above; the greedy (alpha >= n) and norm-weighted (alpha = 1) choices
  are the ones allowed there.
* The SP step decides to stop inside a launch whose grid is larger than the
  GPU holds at once; every workgroup of that launch must still write its rows
  of x.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from checks import assert_close

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def devA(A):
    return dev(np.asarray(A).T).t()


def host(t):
    return t.detach().cpu().numpy()


def banner(msg):
    print(f"[gpu-fullsize] {msg}", flush=True)


# (p, q, n): 80-row slices (one LDS chunk, the rows beyond 16 of the staging
# live); 160-row slices (two chunks of 128 and 32 rows)
RK_SHAPES = [(18000, 2000, 150), (40000, 1000, 120)]


@pytest.fixture(scope="module", params=RK_SHAPES, ids=lambda s: "p%d_q%d_n%d" % s)
def rkprob(request):
    p, q, n = request.param
    banner(f"SP-RK-RGS problem p={p} q={q} n={n}")
    P = W.dense_ils(p, q, n, ratio=0.5, seed=p + q + n)
    return P, devA(P.A), dev(P.b), dev(P.x_star)


@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_rk_fixed_schedule_full_slices(rkprob, form):
    P, A, b, _ = rkprob
    # 2 outer steps of 700 inner steps: 21 whole blocks of 32 and one of 28
    kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=700, seed=5, form=form)
    banner(f"fixed schedule p={P.p} form={form}")
    x, info = ils.rk_solve(A, b, P.p, **kw)
    ref, rinfo = O.rk_solve(P.A, P.b, P.p, **kw)
    assert info.status == ils.OK and info.inner_iters == rinfo.inner_iters == 1400
    assert_close(host(x), ref, 1e-10)


def test_rk_mixed_full_slices(rkprob):
    """FP32 slices of the same heights inside FP64 refinement reach x_ILS."""
    P, A, b, xs = rkprob
    banner(f"mixed converged p={P.p}")
    x, info = ils.rk_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                           stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-8, seed=1)
    assert info.status == ils.OK
    st, x_ils = O.normal_solve(P.A, P.b, P.p)
    assert st == O.OK
    assert_close(host(x), x_ils, 1e-6)


@pytest.fixture(scope="module")
def scdprob():
    # n above the 4096 entries the LDS-resident residual holds; q = 0 keeps
    # the generator cheap (no spectral scaling needed) and A1 well conditioned
    p, n = 5000, 4097
    banner(f"SP-SCD problem p={p} q=0 n={n}")
    P = W.dense_ils(p, 0, n, seed=p + n)
    return P, devA(P.A), dev(P.b)


@pytest.mark.parametrize("alpha,sampling,form", [(10 ** 6, ils.SAMPLE_UNIFORM, ils.FORM_PAPER),
                                                 (1, ils.SAMPLE_NORM, ils.FORM_CORRECTION)],
                         ids=["greedy_paper", "rcd_correction"])
def test_scd_global_residual_path(scdprob, alpha, sampling, form):
    P, A, b = scdprob
    kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=300, seed=6, alpha=alpha,
              sampling=sampling, form=form)
    banner(f"SP-SCD n={P.n} alpha={alpha}")
    x, info = ils.rgs_solve(A, b, P.p, **kw)
    ref, rinfo = O.rgs_solve(P.A, P.b, P.p, **kw)
    assert info.status == ils.OK and info.inner_iters == rinfo.inner_iters == 600
    assert_close(host(x), ref, 1e-10)


def test_scd_uniform_subsets_rejected_above_lds_limit(scdprob):
    P, A, b = scdprob
    _, info = ils.rgs_solve(A, b, P.p, alpha=0, sampling=ils.SAMPLE_UNIFORM)
    assert info.status == ils.ERR_ARG


@pytest.mark.parametrize("form", [ils.FORM_PAPER, ils.FORM_CORRECTION])
def test_sp_deciding_launch_writes_every_row(form):
    """n = 6000: the SP step launches 1500 workgroups, more than are resident
    at once, so some start after the deciding workgroup has published its
    decision.  x is filled with NaN first; every entry must be written, and
    with b = A x* (no noise) the result is x* to the conditioning of A^T J A."""
    p, q, n = 8000, 500, 6000
    banner(f"SP deciding launch p={p} q={q} n={n} form={form}")
    rng = np.random.default_rng(60)
    A1 = rng.standard_normal((p, n))
    A2 = 0.01 * rng.standard_normal((q, n))  # ||A2|| ~ 1.0 against sigma_min(A1) ~ 12
    xs = rng.standard_normal(n)
    A = np.asfortranarray(np.vstack([A1, A2]))
    b = A @ xs
    del A1, A2
    Ad, bd, xsd = devA(A), dev(b), dev(xs)
    del A
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    _, info = ils.sp_solve(Ad, bd, p, out=out, stop_rule=ils.STOP_XREF, x_ref=xsd, tol=1e-9, form=form)
    assert info.status == ils.OK and info.outer_iters >= 2
    xh = host(out)
    assert np.all(np.isfinite(xh))
    assert_close(xh, xs, 1e-8)


# register form of the SCD steps: 4, 8 or 16 entries per thread (n up to
# 1024, 2048, 4096); a full last thread, a ragged one, and the largest n
@pytest.mark.parametrize("n", [1024, 1025, 2049, 4096])
def test_scd_register_form_entry_counts(n):
    p = n + 700
    banner(f"SP-SCD register form n={n}")
    P = W.dense_ils(p, 0, n, seed=n)
    A, b = devA(P.A), dev(P.b)
    for alpha, sampling in ((0, ils.SAMPLE_UNIFORM), (1, ils.SAMPLE_NORM)):
        kw = dict(stop_rule=ils.STOP_FIXED, max_outer=2, max_inner=300, seed=8, alpha=alpha,
                  sampling=sampling, form=ils.FORM_CORRECTION)
        x, info = ils.rgs_solve(A, b, P.p, **kw)
        ref, rinfo = O.rgs_solve(P.A, P.b, P.p, **kw)
        assert info.status == ils.OK and info.inner_iters == rinfo.inner_iters == 600
        assert_close(host(x), ref, 1e-10, what=f"alpha={alpha}")


@pytest.mark.parametrize("shape", [(700, 90, 150), (2600, 300, 1500)])
def test_scd_mixed_fp32_sweeps_reach_x_ils(shape):
    """FP32 A1^T A1 and FP32 inner residual inside FP64 refinement: the
    correction form's fixed point is the FP64 x_ILS."""
    P = W.dense_ils(*shape, ratio=0.5, seed=sum(shape))
    A, b, xs = devA(P.A), dev(P.b), dev(P.x_star)
    x, info = ils.rgs_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                            stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-8, seed=1)
    assert info.status == ils.OK
    st, x_ils = O.normal_solve(P.A, P.b, P.p)
    assert st == O.OK
    assert_close(host(x), x_ils, 1e-6)
