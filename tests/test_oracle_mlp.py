"""Pins for the network reference (CPU only): gradients by back-propagation
against central finite differences, and GELU special values."""
import math

import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.PARAMS == 27668


def test_gelu_closed_forms():
    z = np.array([0.0, 1.0, -1.0, 3.0])
    g = mlp.gelu(z)
    assert g[0] == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15          # Phi(1)
    assert abs(g[2] + 0.15865525393145707) < 1e-15         # -Phi(-1)
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    # derivative by central differences
    h = 1e-6
    for x in (-2.0, -0.3, 0.7, 2.5):
        fd = (mlp.gelu(np.array([x + h]))[0] - mlp.gelu(np.array([x - h]))[0]) / (2 * h)
        assert abs(fd - mlp.gelu_grad(np.array([x]))[0]) < 1e-8


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(3)
    theta = mlp.init(5) + rng.normal(0, 0.01, mlp.PARAMS)
    X = rng.normal(0, 1, (7, mlp.IN))
    T = rng.normal(0, 1, (7, mlp.OUT))
    L, g = mlp.gradients(theta, X, T)
    assert abs(L - mlp.loss(theta, X, T)) < 1e-15
    idx = rng.choice(mlp.PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [0, 66 * 128, 66 * 128 + 128 + 5, mlp.PARAMS - 1]])   # a weight and bias of each kind
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, i


def test_adam_first_step_closed_form():
    """With zero moments the bias corrections cancel at t = 1: m_hat = g and
    v_hat = g^2, so the step is -lr g / (|g| + eps) element by element (a
    swapped b1/b2, a missing bias correction or a wrong sign changes it)."""
    rng = np.random.default_rng(21)
    theta = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50) * np.logspace(-9, 2, 50)
    z = np.zeros(50)
    lr = 3e-3
    t1, m1, v1 = mlp.adam_step(theta, g, z, z, 1, lr)
    np.testing.assert_allclose(t1, theta - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_adam_second_step_hand_worked():
    """Scalar case worked by hand: g1 = 1, g2 = 0.5, lr = 0.1, from zero.
    Step 1: theta1 = -0.1 / (1 + 1e-8).  Step 2: m2 = 0.9 * 0.1 + 0.1 * 0.5
    = 0.14, v2 = 0.999 * 0.001 + 0.001 * 0.25 = 0.001249; m_hat = 0.14 / 0.19
    = 14/19, v_hat = 0.001249 / 0.001999 = 1249/1999, so theta2 = theta1 -
    0.1 * (14/19) / (sqrt(1249/1999) + 1e-8)."""
    th, m, v = mlp.adam_step([0.0], [1.0], [0.0], [0.0], 1, 0.1)
    assert abs(th[0] + 0.1 / (1 + 1e-8)) < 1e-16
    th, m, v = mlp.adam_step(th, [0.5], m, v, 2, 0.1)
    assert abs(m[0] - 0.14) < 1e-15 and abs(v[0] - 0.001249) < 1e-14 * 0.001249
    want = -0.1 / (1 + 1e-8) - 0.1 * (14 / 19) / (math.sqrt(1249 / 1999) + 1e-8)
    assert abs(th[0] - want) < 1e-15
