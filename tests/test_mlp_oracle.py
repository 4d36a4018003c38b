"""Pins of the FP64 MLP oracle: finite differences, closed forms of Adam's
first step and of hand-set networks."""
import numpy as np
import pytest

from oracle import mlp
from paper_2112_10037_amd import gen


def _batch(seed, n=33):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 2, (n, mlp.NF)), rng.uniform(0, 2, n)


def test_layout_size():
    assert mlp.NPARAM == 4801 == gen.mlp_init(0).size


def test_gradient_central_differences():
    x, t = _batch(1)
    theta = gen.mlp_init(3)
    theta[64 * 8:64 * 8 + 64] = 0.05          # nonzero biases so every block is exercised
    _, g = mlp.grad(theta, x, t)
    rng = np.random.default_rng(5)
    idx = np.concatenate([np.arange(0, 8), np.arange(512, 520), np.arange(576, 600),
                          np.arange(4672, 4801), rng.choice(mlp.NPARAM, 200, replace=False)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, x, t) - mlp.loss(tm, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, i


def test_hand_set_network_forward():
    # W1 = [I8; 0], W2 = [I on the first 8; 0], W3 = ones on the first 8, b3 = 0.5:
    # y = 0.5 + sum_f relu(x_f)
    p = {"W1": np.zeros((64, 8)), "b1": np.zeros(64), "W2": np.zeros((64, 64)),
         "b2": np.zeros(64), "W3": np.zeros(64), "b3": np.array([0.5])}
    p["W1"][:8, :8] = np.eye(8)
    p["W2"][:8, :8] = np.eye(8)
    p["W3"][:8] = 1.0
    theta = mlp.pack(p)
    x, _ = _batch(2)
    y, _ = mlp.forward(theta, x)
    assert np.allclose(y, 0.5 + np.maximum(x, 0).sum(axis=1), rtol=0, atol=1e-14)


def test_loss_is_mse():
    theta = mlp.pack({"W1": np.zeros((64, 8)), "b1": np.zeros(64), "W2": np.zeros((64, 64)),
                      "b2": np.zeros(64), "W3": np.zeros(64), "b3": np.array([1.0])})
    x = np.zeros((4, 8))
    t = np.array([0.0, 1.0, 2.0, 3.0])
    assert mlp.loss(theta, x, t) == pytest.approx((1 + 0 + 1 + 4) / 4, abs=0)


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2, so theta1 = theta0 - lr g / (|g| + eps)
    rng = np.random.default_rng(9)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    t1, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(t1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g, v_hat = g^2 at every step
    th, mm, vv = theta, np.zeros(50), np.zeros(50)
    for s in range(1, 6):
        th, mm, vv = mlp.adam_step(th, g, mm, vv, s, lr=1e-3)
    assert np.allclose(th, theta - 5e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)


def test_training_descends():
    # a few hundred full-batch Adam steps on a smooth target lower the loss
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (256, 8))
    t = x[:, 0] * 2 + x[:, 1]
    theta = gen.mlp_init(11)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, x, t)
    for s in range(1, 301):
        _, g = mlp.grad(theta, x, t)
        theta, m, v = mlp.adam_step(theta, g, m, v, s, lr=3e-3)
    assert mlp.loss(theta, x, t) < 0.05 * l0
