"""Pins of the oracle's warm-start network (forward, backward, Adam, bf16 rounding).

The network is the three-layer ReLU perceptron used to map a row sample of b
to the initial value x0 of the SP iteration (SP converges from any x0,
Thm. 2.1).  The pins are: the chain-rule gradient against central finite
differences of the forward loss, forward and backward against torch's
float64 autograd on the CPU (a library routine), a layer that ReLU switches
off entirely (closed form), Adam against torch.optim.Adam and against its
closed form for a constant gradient, and bf16 rounding against torch's
float -> bfloat16 conversion.
"""
import numpy as np
import pytest
import torch

import oracle as O

D_SMALL = (7, 6, 5, 4)


def _params(d, rng, scale=0.5):
    return rng.standard_normal(O.mlp_nparams(d)) * scale


def _split(d, theta):
    out, o = [], 0
    for l in range(3):
        W = theta[o:o + d[l + 1] * d[l]].reshape(d[l + 1], d[l])
        o += d[l + 1] * d[l]
        b = theta[o:o + d[l + 1]]
        o += d[l + 1]
        out.append((W, b))
    return out


def test_nparams_of_the_2000_512_512_1000_network():
    assert O.mlp_nparams((2000, 512, 512, 1000)) == 1_800_168


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    d, B = D_SMALL, 3
    th = _params(d, rng)
    U = rng.standard_normal((d[0], B))
    T = rng.standard_normal((d[3], B))
    loss, g = O.mlp_grad(d, th, U, T)
    assert loss == pytest.approx(O.mlp_loss(d, th, U, T), rel=1e-14)
    h = 1e-6
    fd = np.empty_like(th)
    for k in range(len(th)):
        e = np.zeros_like(th)
        e[k] = h
        fd[k] = (O.mlp_loss(d, th + e, U, T) - O.mlp_loss(d, th - e, U, T)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_forward_and_gradient_match_torch_autograd():
    rng = np.random.default_rng(1)
    d, B = (9, 8, 7, 5), 6
    th = _params(d, rng)
    U = rng.standard_normal((d[0], B))
    T = rng.standard_normal((d[3], B))
    Y, H1, H2 = O.mlp_forward(d, th, U)
    loss, g = O.mlp_grad(d, th, U, T)

    tt = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    layers, o = [], 0
    for l in range(3):
        W = tt[o:o + d[l + 1] * d[l]].view(d[l + 1], d[l])
        o += d[l + 1] * d[l]
        b = tt[o:o + d[l + 1]]
        o += d[l + 1]
        layers.append((W, b))
    h = torch.tensor(U.T)
    for l, (W, b) in enumerate(layers):
        h = torch.nn.functional.linear(h, W, b)
        if l < 2:
            h = torch.relu(h)
    ref = torch.nn.functional.mse_loss(h, torch.tensor(T.T))
    ref.backward()
    np.testing.assert_allclose(Y, h.detach().numpy().T, rtol=1e-13, atol=1e-13)
    assert loss == pytest.approx(ref.item(), rel=1e-13)
    np.testing.assert_allclose(g, tt.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_positive_network_is_an_affine_map():
    """Nonnegative weights, biases and inputs keep every ReLU in its linear
    part, so the network is W3 (W2 (W1 u + b1) + b2) + b3."""
    rng = np.random.default_rng(2)
    d, B = (6, 5, 4, 3), 4
    th = np.abs(_params(d, rng))
    U = np.abs(rng.standard_normal((d[0], B)))
    (W1, b1), (W2, b2), (W3, b3) = _split(d, th)
    expect = W3 @ (W2 @ (W1 @ U + b1[:, None]) + b2[:, None]) + b3[:, None]
    Y, _, _ = O.mlp_forward(d, th, U)
    np.testing.assert_allclose(Y, expect, rtol=1e-14)


def test_switched_off_layer_leaves_only_downstream_biases():
    """With b1 far below zero the first ReLU outputs 0 for every sample, so
    y = W3 relu(b2) + b3 and the gradient of W1, b1 vanishes."""
    rng = np.random.default_rng(3)
    d, B = (6, 5, 4, 3), 4
    th = _params(d, rng)
    (W1, b1), (W2, b2), (W3, b3) = _split(d, th)
    n1 = d[1] * d[0]
    th[n1:n1 + d[1]] = -1e6
    U = rng.standard_normal((d[0], B))
    Y, H1, _ = O.mlp_forward(d, th, U)
    assert np.all(H1 == 0.0)
    expect = W3 @ np.maximum(b2, 0.0) + b3
    np.testing.assert_allclose(Y, np.repeat(expect[:, None], B, axis=1), rtol=1e-14)
    _, g = O.mlp_grad(d, th, U, rng.standard_normal((d[3], B)))
    assert np.all(g[:n1 + d[1]] == 0.0)


def test_loss_of_a_shifted_target():
    rng = np.random.default_rng(4)
    d, B = D_SMALL, 5
    th = _params(d, rng)
    U = rng.standard_normal((d[0], B))
    Y, _, _ = O.mlp_forward(d, th, U)
    assert O.mlp_loss(d, th, U, Y) == 0.0
    assert O.mlp_loss(d, th, U, Y + 0.25) == pytest.approx(0.0625, rel=1e-13)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    n, steps = 50, 7
    w = rng.standard_normal(n)
    m, v = np.zeros(n), np.zeros(n)
    tw = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, steps + 1):
        g = rng.standard_normal(n)
        O.adam_step(w, m, v, g, t, lr=1e-2)
        tw.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(w, tw.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient both bias-corrected moments equal g and g^2
    exactly, so every step is lr * g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    w = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    for t in range(1, 11):
        O.adam_step(w, m, v, g, t, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(w, -10 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.standard_normal(2000) * 10 ** rng.uniform(-6, 6, 2000),
                        [1.0, -1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 0.0, 65504.0]])
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16_round(x), ref)
