"""GPU checks of the autotuner: the sweep picks a valid configuration, the
Gram products launched with the tuned table still match the oracle, and the
saved table reloads to the same choices."""
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


@pytest.mark.parametrize("prec", [ils.PREC_FP64, ils.PREC_MIXED])
def test_tuned_gram_matches_oracle(tmp_path, prec):
    P = W.dense_ils(3000, 300, 200, ratio=0.5, seed=4)
    A = devA(P.A)
    ils.tune_clear()
    try:
        best = ils.tune_gram(A, 0, P.p, precision=prec, reps=3)
        print(f"[gpu-tune] precision {prec}: {best}", flush=True)
        if best["kind"] == ils.GRAM_PERSISTENT:
            assert best["tile"] == 64 and best["workgroups"] == 4
        else:
            assert best["tile"] in (64, 128) and 256 <= best["workgroups"] <= 8192
        assert best["ms"] > 0
        G = ils.gram(A, 0, P.p, precision=prec).cpu().numpy()
        ref = O.gram(P.A, 0, P.p)
        if prec == ils.PREC_FP64:
            assert np.linalg.norm(G - ref) <= 1e-13 * np.linalg.norm(ref)
        else:  # FP32 rounding of the inputs and of a length-p sum
            nrm = np.sqrt((P.A[:P.p] ** 2).sum(axis=0))
            assert np.all(np.abs(G - ref) <= (2 + P.p) * 2.0 ** -24 * np.outer(nrm, nrm))
        f = tmp_path / "tune.json"
        ils.tune_save(f)
        entries = json.loads(f.read_text())["entries"]
        assert len(entries) == 1 and entries[0]["tile"] == best["tile"]
        assert entries[0]["workgroups"] == best["workgroups"] and entries[0]["precision"] == prec
        assert entries[0]["kind"] == best["kind"]
        ils.tune_clear()
        ils.tune_load(f)
        f2 = tmp_path / "tune2.json"
        ils.tune_save(f2)
        assert json.loads(f2.read_text()) == json.loads(f.read_text())
        x, info = ils.sp_solve(A, torch.from_numpy(P.b).cuda(), P.p, stop_rule=ils.STOP_XREF,
                               x_ref=torch.from_numpy(P.x_star).cuda(), tol=1e-9,
                               form=ils.FORM_CORRECTION, precision=prec)
        assert info.status == ils.OK and info.rel_err < 1e-9
    finally:
        ils.tune_clear()


@pytest.mark.parametrize("shape", [(3000, 300, 200), (1500, 200, 1100)], ids=["one_pass_range", "two_pass_only"])
def test_tune_residual_and_its_choices_match_oracle(tmp_path, shape):
    """Every residual launch choice gives A^T J (b - A x) to the oracle's
    value, and the sweep keeps a valid one."""
    p, q, n = shape
    P = W.dense_ils(p, q, n, ratio=0.5, seed=9, spectral="eig")
    A = devA(P.A)
    b = torch.from_numpy(P.b).cuda()
    x = np.random.default_rng(3).standard_normal(n)
    xd = torch.from_numpy(x).cuda()
    ref = O.residual(P.A, P.b, P.p, x)
    ils.tune_clear()
    try:
        best = ils.tune_residual(A, b, P.p, xd, reps=3)
        print(f"[gpu-tune] residual {shape}: {best}", flush=True)
        assert best["kernel"] == "residual" and best["kind"] in (ils.RESID_AUTO, ils.RESID_TWO_PASS)
        assert 64 <= best["workgroups"] <= 2048 and best["ms"] > 0
        r = ils.residual(A, b, P.p, xd).cpu().numpy()
        assert np.linalg.norm(r - ref) <= 1e-12 * np.linalg.norm(ref)
        nb = int(np.ceil(np.log2(n))) if n > 1 else 0
        kb = int(np.ceil(np.log2(p + q)))
        for wg, path in ((128, 0), (512, 0), (1024, 0), (256, 1)):
            ils.tune_clear()
            f = tmp_path / f"r{wg}_{path}.json"
            f.write_text('{"version": 1, "entries": [\n  ' + json.dumps(
                {"kernel": "residual", "precision": 0, "form": 0, "n_bucket": nb, "k_bucket": kb, "tile": 16,
                 "workgroups": wg, "kind": path}) + "\n]}\n")
            ils.tune_load(f)
            r = ils.residual(A, b, P.p, xd).cpu().numpy()
            assert np.linalg.norm(r - ref) <= 1e-12 * np.linalg.norm(ref), (wg, path)
    finally:
        ils.tune_clear()
