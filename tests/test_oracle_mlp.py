"""Pins of the float64 learned-probe-count oracle (oracle/mlp.py): a
hand-worked gradient, central finite differences, the identity network,
Adam's closed form under a constant gradient, bfloat16 rounding against
torch's conversion, and hand cases of the label and probe-count rules."""
import json
import math
import os

import numpy as np
import pytest

from oracle import mlp


def _theta(g):
    return np.concatenate([np.ravel(g["W1"]), g["b1"], np.ravel(g["W2"]), g["b2"], g["w3"],
                           g["b3"]]).astype(np.float64)


def test_handworked_gradient(golden_dir):
    with open(os.path.join(golden_dir, "mlp_2x2_handworked.json")) as f:
        g = json.load(f)
    th = _theta(g)
    *_, yhat = mlp.forward(th, g["X"], g["din"], g["h"])
    assert yhat.tolist() == g["yhat"]
    loss, grad = mlp.loss_and_grad(th, g["X"], g["y"], g["din"], g["h"])
    assert loss == g["loss"]
    np.testing.assert_array_equal(grad, _theta(g["grad"]))


def test_finite_differences():
    rng = np.random.default_rng(5)
    din, h, B = 5, 4, 3
    th = rng.standard_normal(mlp.n_params(din, h))
    X = rng.standard_normal((B, din))
    y = rng.standard_normal(B)
    _, grad = mlp.loss_and_grad(th, X, y, din, h)
    z1, _, z2, _, _ = mlp.forward(th, X, din, h)
    assert np.abs(z1).min() > 1e-3 and np.abs(z2).min() > 1e-3  # away from relu kinks
    hstep = 1e-6
    fd = np.empty_like(th)
    for i in range(len(th)):
        e = np.zeros_like(th)
        e[i] = hstep
        fd[i] = (mlp.loss_and_grad(th + e, X, y, din, h)[0]
                 - mlp.loss_and_grad(th - e, X, y, din, h)[0]) / (2 * hstep)
    np.testing.assert_allclose(grad, fd, rtol=1e-5, atol=1e-8)


def test_identity_network_is_relu():
    din = h = 6
    x = np.array([[1.5, -2.0, 0.0, 3.25, -0.5, 7.0]])
    W1 = np.eye(h)
    W2 = np.eye(h)
    for j in range(h):
        w3 = np.zeros(h)
        w3[j] = 1.0
        th = np.concatenate([W1.ravel(), np.zeros(h), W2.ravel(), np.zeros(h), w3, [0.0]])
        _, h1, _, h2, yhat = mlp.forward(th, x, din, h)
        np.testing.assert_array_equal(h1, np.maximum(x, 0))
        np.testing.assert_array_equal(h2, np.maximum(x, 0))
        assert yhat[0] == max(x[0, j], 0.0)


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step, so each step moves by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, g, m, v, t)
        step = 1e-3 * g / (np.abs(g) + 1e-8)
        np.testing.assert_allclose(th, -t * step, rtol=1e-9, atol=1e-15)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    a = (rng.standard_normal(10000) * np.exp(rng.uniform(-20, 20, 10000))).astype(np.float32)
    a[:4] = [0.0, -0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8]  # ties to even both ways
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(a), ref)
    assert mlp.bf16_round(np.float32([1.0 + 2 ** -8]))[0] == 1.0
    assert mlp.bf16_round(np.float32([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_labels_and_probe_count():
    order = np.array([[4, 2, 9, 1], [7, 3, 5, 0], [1, 0, 2, 3]])
    assert mlp.labels([9, 7, 6], order, 4).tolist() == [3, 1, 4]
    assert mlp.labels([1], order[:1], 3).tolist() == [3]  # beyond the cap
    assert mlp.probe_count([3.0, 3.01, 0.0, -5.0, 20.0], 0.0, 256).tolist() == [8, 9, 1, 1, 256]
    assert mlp.probe_count([2.0], 1.0, 256).tolist() == [8]
    assert mlp.probe_count([math.log2(5)], 0.0, 256).tolist() == [5]


def test_features_and_standardization():
    rng = np.random.default_rng(2)
    xq = rng.standard_normal((50, 8))
    cd = rng.uniform(0, 10, (50, 40))
    F = mlp.features(xq, cd)
    assert F.shape == (50, 8 + mlp.N_DIST)
    np.testing.assert_array_equal(F[:, :8], xq)
    assert np.all(np.diff(F[:, 8:], axis=1) >= 0)
    np.testing.assert_array_equal(F[:, 8:], np.sort(cd, 1)[:, :mlp.N_DIST])
    F[:, 3] = 2.0  # a constant column keeps unit spread
    mean, std = mlp.standardization(F)
    Z = (F - mean) / std
    np.testing.assert_allclose(Z.mean(0), 0, atol=1e-12)
    nz = np.ones(Z.shape[1], bool)
    nz[3] = False
    np.testing.assert_allclose(Z[:, nz].std(0), 1, rtol=1e-12)
    assert std[3] == 1.0
