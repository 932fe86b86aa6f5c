"""GPU parity of the persistent Gram kernel (A1^T A1 and A2^T A2 of Alg. 1
steps 2-3 on per-XCD row ranges with direct global-to-LDS loads) against the
oracle, through the C ABI, on shapes that reach each of its paths: several
tiles with a ragged column tail, a zero-padded last tile, an odd row count
(register tail stage), the bordered two-part product of the paper form with
an odd A1/A2 boundary (register head stage) and q = 0; plus the same shapes
forced onto the split-K kind through a launch table, so both kinds are
checked against the same oracle values.  The FP32 product of the mixed
precision (Sec. 4 remark on single-precision inner work) runs the same
kernel on an FP32 copy of the rows: checked against the FP64 oracle within
the bound of rounding the operands and summing K products in FP32."""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu


def devA(A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to("cuda").t()


def bucket(x):
    b = 0
    while (1 << b) < x:
        b += 1
    return b


def check_gram(G, A, r0, r1):
    ref = O.gram(A, r0, r1)
    Ab = np.abs(A[r0:r1])
    # componentwise: a length-K sum in any order, |err| <= K u |a_i|^T |a_j|
    bound = (r1 - r0) * 2.0 ** -52 * (Ab.T @ Ab) + 1e-300
    assert np.all(np.abs(G - ref) <= bound), np.max(np.abs(G - ref) / bound)
    assert np.linalg.norm(G - ref) <= 1e-13 * np.linalg.norm(ref)


SHAPES = [(3000, 200, 41), (5001, 250, 42), (4096, 513, 43), (20000, 1000, 44)]


def check_gram_f32(G, A, r0, r1):
    ref = O.gram(A, r0, r1)
    Ab = np.abs(A[r0:r1])
    # both operands rounded to FP32 (2 u) and a length-K FP32 sum (K u), u = 2^-24
    bound = (2 + (r1 - r0)) * 2.0 ** -24 * (Ab.T @ Ab) + 1e-300
    assert np.all(np.abs(G - ref) <= bound), np.max(np.abs(G - ref) / bound)
    assert np.allclose(G, G.T, rtol=0, atol=0)


def forced_table(tmp_path, precision, n, K, kind):
    f = tmp_path / "t.json"
    entry = {"kernel": "gram", "precision": precision, "n_bucket": bucket(n), "k_bucket": bucket(K), "tile": 64,
             "workgroups": 4 if kind == ils.GRAM_PERSISTENT else 2048, "kind": kind}
    f.write_text('{"version": 1, "entries": [\n  ' + json.dumps(entry) + "\n]}\n")
    return f


@pytest.mark.parametrize("kind", [ils.GRAM_PERSISTENT, ils.GRAM_SPLITK], ids=["persistent", "splitk"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"K{k}_n{n}" for k, n, _ in SHAPES])
def test_gram_kinds_match_oracle(tmp_path, shape, kind):
    K, n, seed = shape
    A = np.asfortranarray(np.random.default_rng(seed).standard_normal((K, n)))
    Ad = devA(A)
    assert Ad.stride(1) % 2 == 0 or K % 2 == 1
    ils.tune_clear()
    try:
        ils.tune_load(forced_table(tmp_path, ils.PREC_FP64, n, K, kind))
        print(f"[gram-persistent] K={K} n={n} kind={kind}", flush=True)
        G = ils.gram(Ad, 0, K).cpu().numpy()
        check_gram(G, A, 0, K)
    finally:
        ils.tune_clear()


@pytest.mark.parametrize("kind", [ils.GRAM_PERSISTENT, ils.GRAM_SPLITK], ids=["persistent", "splitk"])
@pytest.mark.parametrize("shape", SHAPES + [(18000, 1000, 45)], ids=[f"K{k}_n{n}" for k, n, _ in SHAPES + [(18000, 1000, 45)]])
def test_gram_f32_kinds_match_oracle(tmp_path, shape, kind):
    """FP32 product: the persistent kind reads an FP32 copy (rows padded to a
    multiple of 4, so odd K ends in a register stage); split-K converts while
    staging.  Both within the FP32 bound of the FP64 oracle."""
    K, n, seed = shape
    A = np.asfortranarray(np.random.default_rng(seed).standard_normal((K, n)))
    Ad = devA(A)
    ils.tune_clear()
    try:
        ils.tune_load(forced_table(tmp_path, ils.PREC_MIXED, n, K, kind))
        print(f"[gram-persistent f32] K={K} n={n} kind={kind}", flush=True)
        G = ils.gram(Ad, 0, K, precision=ils.PREC_MIXED).cpu().numpy()
        check_gram_f32(G, A, 0, K)
    finally:
        ils.tune_clear()


def test_gram_f32_offset_rows(tmp_path):
    """Rows [r0, r1) with r0 odd: the copy starts at the range's first row, so
    the FP32 operand is aligned whatever r0 is."""
    K, n = 7003, 300
    A = np.asfortranarray(np.random.default_rng(46).standard_normal((K, n)))
    Ad = devA(A)
    ils.tune_clear()
    try:
        ils.tune_load(forced_table(tmp_path, ils.PREC_MIXED, n, K - 3, ils.GRAM_PERSISTENT))
        print(f"[gram-persistent f32] rows 3..{K} n={n}", flush=True)
        G = ils.gram(Ad, 3, K, precision=ils.PREC_MIXED).cpu().numpy()
        check_gram_f32(G, A, 3, K)
    finally:
        ils.tune_clear()


def test_mixed_sp_with_f32_persistent_gram(tmp_path):
    """Mixed SP (correction form) with the FP32 Gram taken from the copy: the
    refined iterate reaches the FP64 oracle's solution."""
    p, q, n = 12000, 4000, 400
    P = W.dense_ils(p, q, n, ratio=0.5, seed=47, spectral="eig")
    A = devA(P.A)
    b = torch.from_numpy(P.b).cuda()
    ils.tune_clear()
    try:
        ils.tune_load(forced_table(tmp_path, ils.PREC_MIXED, n, p, ils.GRAM_PERSISTENT))
        print(f"[gram-persistent f32] mixed SP p={p} q={q} n={n}", flush=True)
        x, info = ils.sp_solve(A, b, P.p, precision=ils.PREC_MIXED, form=ils.FORM_CORRECTION,
                               stop_rule=ils.STOP_XREF, x_ref=torch.from_numpy(P.x_star).cuda(), tol=1e-11)
    finally:
        ils.tune_clear()
    xs = O.normal_solve(P.A, P.b, P.p)[1]
    assert info.status == ils.OK
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("pq", [(4001, 999), (18001, 1999), (3000, 0)], ids=["odd_p", "odd_p_large", "q0"])
def test_two_part_bordered_product_in_sp(pq):
    """The paper form's one-launch bordered products [A1 b1], [A2 b2]: the
    first SP iterate from x0 = 0 is x1 = (A1^T A1)^{-1} A^T J b (eq. Sec23),
    and later iterates follow B x_k + c; compared with the oracle after 3
    fixed steps."""
    p, q = pq
    n = 300
    P = W.dense_ils(p, q, n, ratio=0.5, seed=p + q, spectral="eig")
    A = devA(P.A)
    b = torch.from_numpy(P.b).cuda()
    print(f"[gram-persistent] SP p={p} q={q} n={n}", flush=True)
    x, info = ils.sp_solve(A, b, P.p, stop_rule=ils.STOP_FIXED, max_outer=3)
    ref, rinfo = O.sp_solve(P.A, P.b, P.p, stop_rule=O.STOP_FIXED, max_outer=3)
    assert info.status == ils.OK and info.outer_iters == rinfo.outer_iters == 3
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.all(np.abs(xh - ref) <= 1e-9 * np.abs(ref).max())


def test_unaligned_rows_fall_back():
    """A row range that starts at an odd row has 8-byte aligned columns only:
    the launch takes the split-K kernel, and the product is still exact."""
    A = np.asfortranarray(np.random.default_rng(7).standard_normal((6001, 260)))
    Ad = devA(A)
    G = ils.gram(Ad, 1, 6001).cpu().numpy()
    check_gram(G, A, 1, 6001)


def test_resident_gram_is_reproducible(tmp_path):
    # the resident launch reorders wave issue by arrival rank (counters that
    # the reduction clears after each launch): the products and their order
    # of summation are fixed, so repeated launches, here with a resident
    # launch of the FP32 kind in between, give the same bits
    K, n = 20000, 1000
    A = np.random.default_rng(45).standard_normal((K, n))
    f = tmp_path / "t.json"
    entries = [{"kernel": "gram", "precision": prec, "n_bucket": bucket(n), "k_bucket": bucket(K), "tile": 64,
                "workgroups": 4, "kind": ils.GRAM_PERSISTENT} for prec in (ils.PREC_FP64, ils.PREC_MIXED)]
    f.write_text('{"version": 1, "entries": [\n  ' + ",\n  ".join(json.dumps(e) for e in entries) + "\n]}\n")
    ils.tune_clear()
    try:
        ils.tune_load(f)
        dA = devA(A)
        G0 = ils.gram(dA, 0, K).cpu().numpy()
        ils.gram(dA, 0, K, precision=ils.PREC_MIXED)
        G1 = ils.gram(dA, 0, K).cpu().numpy()
        G2 = ils.gram(dA, 0, K).cpu().numpy()
        assert np.array_equal(G0, G1) and np.array_equal(G0, G2)
        check_gram(G0, A, 0, K)
    finally:
        ils.tune_clear()
