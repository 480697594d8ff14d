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
