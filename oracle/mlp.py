"""FP64 reference of the warm-start network (test infrastructure only).

The network maps (T/Tc, R, r/R) of a droplet to the density at radius r:
three inputs, three hidden layers of 64 tanh units, one linear output
(the density in units of the critical density).  Inputs are normalised as
x1 = (T/Tc - 0.8)/0.15, x2 = (R - 47.5)/32.5, x3 = r/R - 1.

Flat parameter vector (8641 values), in this order:
  W1[64][3], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[1][64], b4[1]
(row-major, W_l maps layer l-1 to layer l as h_l = tanh(W_l h_{l-1} + b_l)).

Loss: mean squared error over the batch.  Optimiser: Adam with bias
correction (beta1 0.9, beta2 0.999, eps 1e-8).
"""
from __future__ import annotations

import numpy as np

H = 64
SHAPES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
          ("W3", (H, H)), ("b3", (H,)), ("W4", (1, H)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == NPARAM
    out, k = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = theta[k:k + n].reshape(shp)
        k += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def normalise(X):
    X = np.asarray(X, dtype=np.float64)
    Z = np.empty_like(X)
    Z[:, 0] = (X[:, 0] - 0.8) / 0.15
    Z[:, 1] = (X[:, 1] - 47.5) / 32.5
    Z[:, 2] = X[:, 2] - 1.0
    return Z


def forward(theta, X, keep=False):
    """Network output y[n] for raw inputs X[n, 3]."""
    p = unpack(theta)
    a0 = normalise(X)
    h1 = np.tanh(a0 @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    h3 = np.tanh(h2 @ p["W3"].T + p["b3"])
    y = (h3 @ p["W4"].T + p["b4"])[:, 0]
    if keep:
        return y, (a0, h1, h2, h3)
    return y


def loss(theta, X, Y):
    y = forward(theta, X)
    return float(np.mean((y - np.asarray(Y, dtype=np.float64)) ** 2))


def grad(theta, X, Y):
    """Gradient of the mean squared error with respect to the flat parameters."""
    p = unpack(theta)
    y, (a0, h1, h2, h3) = forward(theta, X, keep=True)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(Y, dtype=np.float64)) / n          # dL/dy
    g = {}
    g["W4"] = dy[None, :] @ h3
    g["b4"] = np.array([dy.sum()])
    d3 = (dy[:, None] @ p["W4"]) * (1.0 - h3 ** 2)                 # dL/d(pre-activation 3)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ a0
    g["b1"] = d1.sum(0)
    return pack(g)


def adam_step(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at iteration t (1-based).  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(theta, X, Y, iters, lr=1e-3):
    """Full-batch Adam; returns (theta, loss history)."""
    theta = np.array(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, iters + 1):
        hist.append(loss(theta, X, Y))
        theta, m, v = adam_step(theta, m, v, grad(theta, X, Y), t, lr)
    return theta, hist
