"""ils_residual_noalloc (the residual r = A^T J (b - A x) of eq. Sec12 with the
library's fixed device workspace) against ils_residual, through the C ABI:
several calls in a row on one handle, each smaller than the one before, with
both the one-pass (n <= 1024) and the two-pass (n > 1024) kernels; plus the
size limit and argument errors, which return before any launch."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import paper_2203_15340_amd as ils
import workloads as W

pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = 1 << 20


def _dev(P):
    import torch
    A = torch.from_numpy(np.ascontiguousarray(P.A.T)).cuda().t()
    b = torch.from_numpy(P.b).cuda()
    return A, b


def _call(L, h, A, b, p, x, r, fn):
    m, n = A.shape
    return getattr(L, fn)(h, p, m - p, n, C.c_void_p(A.data_ptr()), A.stride(1), C.c_void_p(b.data_ptr()),
                          C.c_void_p(x.data_ptr()), C.c_void_p(r.data_ptr()))


def test_noalloc_residual_matches_allocating_entry_point():
    import torch
    L = ils.load_library()
    h = ils.handle(torch.device("cuda", 0))
    shapes = [(18000, 2000, 1000, 11), (2400, 700, 1100, 12), (700, 90, 150, 13), (64, 0, 7, 14)]
    for (p, q, n, seed) in shapes:
        P = W.dense_ils(p, q, n, ratio=0.5, seed=seed, spectral="eig")
        A, b = _dev(P)
        x = torch.from_numpy(np.random.default_rng(seed).standard_normal(n)).cuda()
        r_ref = torch.empty(n, dtype=torch.float64, device="cuda")
        r_new = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        print(f"noalloc residual p={p} q={q} n={n}", flush=True)
        assert _call(L, h, A, b, p, x, r_ref, "ils_residual") == ils.OK
        assert _call(L, h, A, b, p, x, r_new, "ils_residual_noalloc") == ils.OK
        torch.cuda.synchronize()
        # the same kernels on the same inputs: the same sums in the same order
        assert torch.equal(r_new, r_ref), (p, q, n)
        ro = O.residual(P.A, P.b, p, x.cpu().numpy())
        rn = r_new.cpu().numpy()
        assert np.linalg.norm(rn - ro) <= 1e-10 * np.linalg.norm(ro), (p, q, n)
        assert np.all(np.abs(rn - ro) <= 1e-10 * (np.abs(P.A).T @ (np.abs(P.b) + np.abs(P.A) @ np.abs(
            x.cpu().numpy())))), (p, q, n)


def test_noalloc_residual_limits_and_errors():
    import torch
    L = ils.load_library()
    h = ils.handle(torch.device("cuda", 0))
    A = torch.zeros(4, 2, dtype=torch.float64, device="cuda")
    v = torch.zeros(4, dtype=torch.float64, device="cuda")
    Ap, vp = C.c_void_p(A.data_ptr()), C.c_void_p(v.data_ptr())
    # workspace above the fixed 2^20 doubles: rejected before any launch
    m = SCRATCH_DOUBLES - 256 * 1000 + 1
    assert L.ils_residual_noalloc(h, m, 0, 1000, Ap, m, vp, vp, vp) == ils.ERR_ARG
    m = SCRATCH_DOUBLES  # two-pass path (n > 1024) needs at least 2 m
    assert L.ils_residual_noalloc(h, m, 0, 2000, Ap, m, vp, vp, vp) == ils.ERR_ARG
    assert L.ils_residual_noalloc(None, 4, 0, 2, Ap, 4, vp, vp, vp) == ils.ERR_ARG
    assert L.ils_residual_noalloc(h, 4, 0, 2, Ap, 3, vp, vp, vp) == ils.ERR_ARG
    assert L.ils_residual_noalloc(h, 4, 0, 0, Ap, 4, vp, vp, vp) == ils.ERR_ARG
    assert L.ils_residual_noalloc(h, 4, 0, 2, None, 4, vp, vp, vp) == ils.ERR_ARG
