"""Pins of the FP64 MLP reference: gradients against central finite
differences, closed forms for the output layer, and Adam's first step."""
import numpy as np

from oracle import mlp_ref as M

F = 24


def rand_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(M.num_params(F)) * scale


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    p = rand_params(1)
    X = rng.standard_normal((7, F))
    T = rng.standard_normal(7)
    L, g = M.loss_and_grad(p, X, T)
    idx = rng.choice(len(p), 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num = (M.loss(p + e, X, T) - M.loss(p - e, X, T)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])), i


def test_output_layer_closed_form():
    # with every hidden unit switched off, y = b3 and only b3 gets a gradient
    p = np.zeros(M.num_params(F))
    w = M.unpack(p, F)
    w["b1"][:] = -1.0
    w["b3"][:] = 0.5
    p = M.pack(w, F)
    X = np.ones((3, F))
    T = np.array([0.0, 1.0, 2.0])
    L, g = M.loss_and_grad(p, X, T)
    assert abs(L - np.mean((0.5 - T) ** 2)) < 1e-15
    gd = M.unpack(g, F)
    assert abs(gd["b3"][0] - np.mean(2 * (0.5 - T))) < 1e-15
    assert np.all(gd["W1"] == 0) and np.all(gd["W2"] == 0) and np.all(gd["w3"] == 0)


def test_single_unit_chain_rule():
    # one active unit per layer: y = w3_0 * relu(W2_00 * relu(W1_0 . x + b1_0) + b2_0) + b3
    p = np.zeros(M.num_params(F))
    w = M.unpack(p, F)
    w["W1"][0, 0], w["b1"][0] = 2.0, 0.5
    w["W2"][0, 0], w["b2"][0] = 1.5, 0.25
    w["w3"][0], w["b3"][0] = -0.75, 0.1
    p = M.pack(w, F)
    x = np.zeros((1, F))
    x[0, 0] = 0.3
    y, _ = M.forward(p, x)
    h1 = 2.0 * 0.3 + 0.5
    h2 = 1.5 * h1 + 0.25
    assert abs(y[0] - (-0.75 * h2 + 0.1)) < 1e-15
    L, g = M.loss_and_grad(p, x, np.array([0.0]))
    gd = M.unpack(g, F)
    dy = 2 * y[0]
    assert abs(gd["w3"][0] - dy * h2) < 1e-14
    assert abs(gd["W2"][0, 0] - dy * -0.75 * h1) < 1e-14
    assert abs(gd["W1"][0, 0] - dy * -0.75 * 1.5 * 0.3) < 1e-14


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = M.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # with bias correction the first step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
