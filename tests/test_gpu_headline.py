"""Parity at the benchmark's own size and launch configuration: A1 18000 x
1000, A2 2000 x 1000 (Gaussian, ||A2|| = 0.5 sigma_min(A1)), FP64 SP to a
relative error of 1e-6, with the committed MI355X Gram launch table loaded as
the benchmark loads it (64-tiles, 24 K-slices for A1).  The whole solve is
compared with the FP64 oracle (it finishes in about a second at this size),
and entries of the two Gram products, sampled at tile and slice boundaries,
with dot products of the columns computed one by one."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from checks import assert_close

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu

TUNE = os.path.join(os.path.dirname(ils.__file__), "tune", "gram_mi355x.json")


@pytest.fixture(scope="module")
def big():
    print("[gpu-headline] generating A1 18000x1000 + A2 2000x1000", flush=True)
    P = W.large(ratio=0.5, seed=1)
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    b = torch.from_numpy(P.b).cuda()
    xs = torch.from_numpy(P.x_star).cuda()
    ils.tune_load(TUNE)
    try:
        yield P, A, b, xs
    finally:
        ils.tune_clear()


def test_headline_solve_matches_oracle(big):
    P, A, b, xs = big
    x, info = ils.sp_solve(A, b, P.p, stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6)
    ref, rinfo = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-6)
    assert info.status == ils.OK and rinfo.status == O.OK
    assert info.outer_iters == rinfo.outer_iters
    assert_close(x.cpu().numpy(), ref, 1e-10)
    assert info.rel_err < 1e-6
    assert info.rel_err == pytest.approx(rinfo.rel_err, rel=1e-6)


def test_headline_correction_form_matches_oracle(big):
    P, A, b, xs = big
    kw = dict(stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6, form=ils.FORM_CORRECTION)
    x, info = ils.sp_solve(A, b, P.p, **kw)
    ref, rinfo = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-6,
                            form=O.FORM_CORRECTION)
    assert info.status == ils.OK and rinfo.status == O.OK
    assert info.outer_iters == rinfo.outer_iters
    assert_close(x.cpu().numpy(), ref, 1e-10)


def test_headline_ratio_09_matches_oracle():
    """The slower-converging variant of the same problem (||A2|| = 0.9
    sigma_min(A1)): same outer count as the oracle, iterates to 1e-10."""
    P = W.large(ratio=0.9, seed=1)
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    b, xs = torch.from_numpy(P.b).cuda(), torch.from_numpy(P.x_star).cuda()
    ils.tune_load(TUNE)
    try:
        x, info = ils.sp_solve(A, b, P.p, stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-6)
    finally:
        ils.tune_clear()
    ref, rinfo = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_XREF, x_ref=P.x_star, tol=1e-6)
    assert info.status == ils.OK and rinfo.status == O.OK
    assert info.outer_iters == rinfo.outer_iters
    assert_close(x.cpu().numpy(), ref, 1e-10)


def _sample_pairs(n, rng, count=48):
    # tile edges (64-column tiles), the last column, and random pairs
    edges = [0, 1, 63, 64, 127, 128, 511, 512, 959, 960, n - 2, n - 1]
    pairs = [(i, j) for i in edges for j in edges if i >= j]
    pairs += [tuple(sorted(rng.integers(0, n, size=2), reverse=True)) for _ in range(count)]
    return pairs


@pytest.mark.parametrize("part", ["A1", "A2"])
def test_headline_gram_sampled_entries(big, part):
    P, A, _, _ = big
    r0, r1 = (0, P.p) if part == "A1" else (P.p, P.m)
    G = ils.gram(A, r0, r1).cpu().numpy()
    assert np.array_equal(G, G.T)
    Ah = np.asarray(P.A)[r0:r1]
    norms = np.linalg.norm(Ah, axis=0)
    for i, j in _sample_pairs(P.n, np.random.default_rng(5)):
        exact = float(np.dot(Ah[:, i], Ah[:, j]))
        # FP64 sums of r1 - r0 products: a few units of rounding times the scale
        assert abs(G[i, j] - exact) <= 1e-13 * norms[i] * norms[j], (part, i, j)


def test_headline_mixed_correction_reaches_x_ils(big):
    """Mixed precision at the benchmark's size with the committed table's FP32
    entry for A1 18000 x 1000: FP32 Gram of A1, FP64 elimination and FP64
    residual A^T J (b - A x_k).  The correction form's fixed point is x_ILS
    whatever the FP32 error in A1^T A1, so the result is checked against the
    FP64 normal-equation solution, normwise and componentwise."""
    P, A, b, xs = big
    x, info = ils.sp_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                           stop_rule=ils.STOP_XREF, x_ref=xs, tol=1e-8)
    assert info.status == ils.OK
    st, x_ils = O.normal_solve(P.A, P.b, P.p)
    assert st == O.OK
    assert_close(x.cpu().numpy(), x_ils, 1e-6)
