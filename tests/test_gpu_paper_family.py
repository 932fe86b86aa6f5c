"""The paper's experiment family (Sec. 5: A1 = U[0,1) p x n, A2 = 7 eye(q, n),
b = U[0,1), x0 = 0, stop at RR < 1e-6) at a reduced size, GPU against the
oracle: same outer count (the paper reports one SP step for this family) and
iterates to 1e-10.  The reduced size keeps p / n large enough that
A1^T A1 - 49 I stays positive definite, as at the paper's sizes."""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu


def devA(A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A).T)).to("cuda").t()


@pytest.mark.parametrize("shape", [(4000, 1000, 1000), (5000, 1, 1300)],
                         ids=["q_eq_n", "minkowski_q1"])
def test_sp_on_paper_family(shape):
    p, q, n = shape
    P = W.paper_family(p, q, n, seed=7)
    print(f"[gpu-paper] p={p} q={q} n={n}", flush=True)
    A, b = devA(P.A), torch.from_numpy(P.b).cuda()
    x, info = ils.sp_solve(A, b, p, stop_rule=ils.STOP_RR, tol=1e-6)
    ref, rinfo = O.sp_solve(P.A, P.b, p, stop_rule=O.STOP_RR, tol=1e-6, variant=O.SP_EXPLICIT)
    assert info.status == ils.OK and rinfo.status == O.OK
    assert info.outer_iters == rinfo.outer_iters
    assert info.rr < 1e-6
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - ref) / np.linalg.norm(ref) < 1e-10
