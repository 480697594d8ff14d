"""Float64 reference of the threshold-bracket network (66 -> 128 -> 128 -> 20,
exact GELU on the hidden layers, linear output, mean-squared-error loss).

TEST INFRASTRUCTURE ONLY: used to check the GPU forward pass, gradients and
the Adam update.
Parameter vector layout: W1 [66][128], b1 [128], W2 [128][128], b2 [128],
W3 [128][20], b3 [20], row-major (W[i][o] at i * O + o).
"""
import math

import numpy as np

IN, H, OUT = 66, 128, 20
SIZES = [("W1", (IN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, OUT)), ("b3", (OUT,))]
PARAMS = sum(int(np.prod(s)) for _, s in SIZES)

_erf = np.vectorize(math.erf)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X):
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ p["W1"] + p["b1"]
    A1 = gelu(Z1)
    Z2 = A1 @ p["W2"] + p["b2"]
    A2 = gelu(Z2)
    Y = A2 @ p["W3"] + p["b3"]
    return Y, (X, Z1, A1, Z2, A2)


def loss(theta, X, T):
    Y, _ = forward(theta, X)
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def gradients(theta, X, T):
    """(loss, gradient vector) by back-propagation."""
    p = unpack(theta)
    Y, (X, Z1, A1, Z2, A2) = forward(theta, X)
    T = np.asarray(T, dtype=np.float64)
    n = Y.size
    dY = 2.0 * (Y - T) / n
    g = {"W3": A2.T @ dY, "b3": dY.sum(0)}
    dZ2 = (dY @ p["W3"].T) * gelu_grad(Z2)
    g["W2"] = A1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ p["W2"].T) * gelu_grad(Z1)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(0)
    vec = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return float(np.mean((Y - T) ** 2)), vec


def init(seed):
    """He-uniform weights (float64) for tests; biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / shape[0])
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, "Adam: a method for stochastic
    optimization", ICLR 2015, Algorithm 1) in float64 at step t >= 1:
      m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,
      m_hat = m / (1 - b1^t),   v_hat = v / (1 - b2^t),
      theta <- theta - lr m_hat / (sqrt(v_hat) + eps).
    Returns (theta, m, v) as new arrays."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
