"""GPU checks of the learned warm start (ils_ws_*): BF16 forward and backward
against the oracle's FP64 network on the same bf16-rounded weights and
inputs, Adam against the oracle's Adam, and what a trained network gains
over the zero start inside SP (Thm. 2.1: SP converges from any x0, so the
network can only change the number of outer steps).

Tolerance for forward and gradients: 2e-2 relative (Frobenius, per
parameter block).  The GPU rounds the hidden activations and the back-
propagated errors to bf16 (unit roundoff 2^-9); the oracle keeps them in
FP64, so each layer adds a relative error of a few 1e-3.
The gain over the zero start is measured, not pinned.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

torch = pytest.importorskip("torch")
import paper_2203_15340_amd as ils  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def banner(msg):
    print(f"[gpu-ws] {msg}", flush=True)


def bf16(a):
    return torch.as_tensor(a).to(torch.bfloat16).to(torch.float64).numpy()


def blocks(d):
    out, o = [], 0
    for l in range(3):
        out.append((f"W{l + 1}", o, o + d[l + 1] * d[l]))
        o += d[l + 1] * d[l]
        out.append((f"b{l + 1}", o, o + d[l + 1]))
        o += d[l + 1]
    return out


def frel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# (m, n, d_in stride, hidden, batch): ragged small network, the 2000-512-512-1000 one
NETS = [(300, 70, 6, 40, 13), (20000, 1000, 10, 512, 37)]


@pytest.fixture(scope="module", params=NETS, ids=lambda c: "m%d_n%d_h%d_b%d" % (c[0], c[1], c[3], c[4]))
def net(request):
    m, n, stride, hidden, batch = request.param
    rows = np.arange(0, m, stride)
    banner(f"network {len(rows)}-{hidden}-{hidden}-{n}, batch {batch}")
    ws = ils.WarmStart(m, n, rows, hidden=hidden, seed=11)
    d = (len(rows), hidden, hidden, n)
    rng = np.random.default_rng(m + hidden)
    th = ws.get_params().cpu().numpy().astype(np.float64)
    for name, a, b in blocks(d):
        if name.startswith("b"):
            th[a:b] = 0.1 * rng.standard_normal(b - a)
    th = bf16(th)
    ws.set_params(torch.from_numpy(th.astype(np.float32)).to(DEV))
    U = bf16(rng.standard_normal((d[0], batch)))
    T = rng.standard_normal((d[3], batch)).astype(np.float32).astype(np.float64)
    yield ws, d, th, U, T
    ws.close()


def test_init_and_params_roundtrip(net):
    ws, d, th, _, _ = net
    assert ws.nparams == O.mlp_nparams(d)
    np.testing.assert_array_equal(ws.get_params().cpu().numpy(), th.astype(np.float32))


def test_forward_matches_oracle(net):
    ws, d, th, U, _ = net
    Y = ws.forward(torch.from_numpy(U.astype(np.float32)).to(DEV)).cpu().numpy()
    ref, _, _ = O.mlp_forward(d, th, U)
    assert frel(Y, ref) < 2e-2


def test_gradient_matches_oracle(net):
    ws, d, th, U, T = net
    loss, g = ws.grad(torch.from_numpy(U.astype(np.float32)).to(DEV),
                      torch.from_numpy(T.astype(np.float32)).to(DEV))
    g = g.cpu().numpy().astype(np.float64)
    rloss, rg = O.mlp_grad(d, th, U, T)
    assert loss == pytest.approx(rloss, rel=2e-2)
    for name, a, b in blocks(d):
        e = frel(g[a:b], rg[a:b])
        banner(f"{name}: relative error {e:.2e}")
        assert e < 2e-2, name
        cos = float(g[a:b] @ rg[a:b] / (np.linalg.norm(g[a:b]) * np.linalg.norm(rg[a:b])))
        assert cos > 0.999, name


def test_adam_matches_oracle(net):
    ws, d, th, _, _ = net
    rng = np.random.default_rng(5)
    w = th.copy()
    m1, m2 = np.zeros_like(w), np.zeros_like(w)
    ws.set_params(torch.from_numpy(th.astype(np.float32)).to(DEV))
    for t in (1, 2, 3):
        g = (rng.standard_normal(len(w)) * 10.0 ** rng.uniform(-4, 0, len(w))).astype(np.float32)
        ws.adam(torch.from_numpy(g).to(DEV), lr=1e-3)
        O.adam_step(w, m1, m2, g.astype(np.float64), t, lr=1e-3)
    got = ws.get_params().cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - w) / (1e-3 + np.abs(w))) < 1e-5
    ws.set_params(torch.from_numpy(th.astype(np.float32)).to(DEV))


@pytest.fixture(scope="module")
def family():
    """A small shared-A family: p=500, q=100, n=50; solutions in a random
    4-dimensional subspace plus 1e-3 noise; the network sees every 5th row."""
    P = W.dense_ils(500, 100, 50, ratio=0.7, seed=21)
    U, _ = np.linalg.qr(np.random.default_rng(22).standard_normal((50, 4)))
    Xtr = W.planted_columns(50, 4096, seed=23, basis=U, noise=1e-3)
    Xte = W.planted_columns(50, 256, seed=24, basis=U, noise=1e-3)

    def dv(M):
        return torch.from_numpy(np.ascontiguousarray(M.T)).to(DEV).t()
    return P, dv(P.A), dv(P.A @ Xtr), dv(Xtr), dv(P.A @ Xte), dv(Xte), Xte


def test_training_lowers_loss_and_sp_steps(family, tmp_path):
    P, A, Btr, Xtr, Bte, Xte_d, Xte = family
    ws = ils.WarmStart(P.m, P.n, np.arange(0, P.m, 5), hidden=64, seed=3)
    first = ws.train(Btr, Xtr, epochs=1, batch=256, lr=2e-3)
    last = ws.train(Btr, Xtr, epochs=40, batch=256, lr=2e-3)
    banner(f"training loss {first:.3e} -> {last:.3e}")
    assert np.isfinite(last) and last < 0.2 * first
    X0 = ws.infer(Bte)
    init_err = np.linalg.norm(X0.cpu().numpy() - Xte, axis=0) / np.linalg.norm(Xte, axis=0)
    banner(f"warm-start initial relative error: median {np.median(init_err):.3e}")
    assert np.median(init_err) < 0.3
    kw = dict(stop_rule=ils.STOP_XREF, tol=1e-6, x_ref=Xte_d)
    _, iz, itz = ils.sp_solve_multi(A, Bte, P.p, **kw)
    Xw, iw, itw = ils.sp_solve_multi(A, Bte, P.p, X0=X0, **kw)
    assert iz.status == iw.status == ils.OK
    banner(f"mean outer steps: zero start {itz.mean():.2f}, warm start {itw.mean():.2f}")
    assert itw.mean() < itz.mean()
    assert iw.rel_err < 1e-6
    # save / load round trip reproduces the same estimates
    path = tmp_path / "ws.bin"
    ws.save(path)
    ws2 = ils.WarmStart(P.m, P.n, np.arange(0, P.m, 5), hidden=64, seed=99)
    ws2.load(path)
    assert torch.equal(ws2.infer(Bte), X0)
    ws2.close()
    ws.close()


def test_argument_errors():
    with pytest.raises(ils.ILSError):
        ils.WarmStart(100, 10, np.array([0, 100]), hidden=8)
    with pytest.raises(ils.ILSError):
        ils.WarmStart(100, 10, np.array([], dtype=np.int64), hidden=8)
