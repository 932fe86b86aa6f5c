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
        assert best["tile"] in (64, 128) and 256 <= best["workgroups"] <= 8192 and best["ms"] > 0
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
