"""FP64 reference of the warm-start network (oracle; test infrastructure only).

26 -> 64 -> 64 -> 1 with SiLU, h = silu(x W + b). Parameter vector (the
library's layout): W1 (26 x 64, input-major), b1 (64), W2 (64 x 64), b2 (64),
W3 (64), b3 (1). Loss: mean squared error. Optimiser: Adam (Kingma & Ba,
"Adam: a method for stochastic optimization", 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

NIN, NH = 26, 64
SIZES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)),
         ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def _sig(a):
    return 1.0 / (1.0 + np.exp(-a))


def forward(theta, X, cache=False):
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ p["W1"] + p["b1"]
    h1 = a1 * _sig(a1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = a2 * _sig(a2)
    y = h2 @ p["W3"] + p["b3"][0]
    if cache:
        return y, (X, a1, h1, a2, h2)
    return y


def loss_grad(theta, X, t):
    """L = mean((y - t)^2) and dL/dtheta by the chain rule."""
    p = unpack(theta)
    y, (X, a1, h1, a2, h2) = forward(theta, X, cache=True)
    m = len(y)
    e = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(e * e))
    dy = 2.0 * e / m
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    s2 = _sig(a2)
    da2 = np.outer(dy, p["W3"]) * (s2 * (1 + a2 * (1 - s2)))
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(0)
    s1 = _sig(a1)
    da1 = (da2 @ p["W2"].T) * (s1 * (1 + a1 * (1 - s1)))
    g["W1"] = X.T @ da1
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; step counts from 1. Returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(rng, scale=1.0):
    """He-style random initialisation (the caller's random numbers)."""
    d = {"W1": rng.standard_normal((NIN, NH)) * scale * np.sqrt(2.0 / NIN),
         "b1": np.zeros(NH),
         "W2": rng.standard_normal((NH, NH)) * scale * np.sqrt(2.0 / NH),
         "b2": np.zeros(NH),
         "W3": rng.standard_normal(NH) * scale * np.sqrt(1.0 / NH),
         "b3": np.zeros(1)}
    return pack(d)
