"""Rank-predictor MLP, plain NumPy in float64 (oracle side; test infrastructure only).

Not part of the paper: the predictor is a project extension that sizes the randomized sketch of
each box's interpolative decomposition (Def. 3.1, Sec. 3.2) before the column-pivoted QR decides
the rank.  What the GPU path computes, written out directly:

  xn = (x - mu) / sd
  h1 = tanh(W1 xn + b1)        W1: 64 x 16
  h2 = tanh(W2 h1 + b2)        W2: 64 x 64
  y  = W3 . h2 + b3            the predicted log(rank)

  pinball loss at quantile tau, r = t - y:  L = sum_b (tau r_b if r_b > 0 else (tau - 1) r_b)

Parameters are one flat vector in the order mu[16], sd[16], W1 (row-major), b1, W2 (row-major),
b2, W3, b3.  The gradient is backpropagation written step by step; finite differences pin it.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 16, 64
SIZES = [("mu", N_IN), ("sd", N_IN), ("W1", N_H * N_IN), ("b1", N_H), ("W2", N_H * N_H), ("b2", N_H),
         ("W3", N_H), ("b3", 1)]
N_PARAM = sum(n for _, n in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, n in SIZES:
        out[name] = p[o:o + n]
        o += n
    out["W1"] = out["W1"].reshape(N_H, N_IN)
    out["W2"] = out["W2"].reshape(N_H, N_H)
    out["b3"] = out["b3"][0]
    return out


def pack(d):
    parts = []
    for name, n in SIZES:
        parts.append(np.atleast_1d(np.asarray(d[name], dtype=np.float64)).reshape(-1))
    p = np.concatenate(parts)
    assert p.size == N_PARAM
    return p


def forward(p, x, keep=False):
    """Predicted log(rank) of every row of x (n x 16)."""
    d = unpack(p)
    xn = (np.asarray(x, dtype=np.float64) - d["mu"]) / d["sd"]
    h1 = np.tanh(xn @ d["W1"].T + d["b1"])
    h2 = np.tanh(h1 @ d["W2"].T + d["b2"])
    y = h2 @ d["W3"] + d["b3"]
    if keep:
        return y, (xn, h1, h2)
    return y


def pinball(y, t, tau):
    r = np.asarray(t, dtype=np.float64) - y
    return float(np.sum(np.where(r > 0, tau * r, (tau - 1.0) * r)))


def loss(p, x, t, tau):
    return pinball(forward(p, x), t, tau)


def grad(p, x, t, tau):
    """Gradient of the summed pinball loss with respect to p (zero for mu, sd)."""
    d = unpack(p)
    y, (xn, h1, h2) = forward(p, x, keep=True)
    r = np.asarray(t, dtype=np.float64) - y
    dy = np.where(r > 0, -tau, 1.0 - tau)                  # dL/dy per sample
    g = {name: np.zeros(n) for name, n in SIZES}
    g["W3"] = dy @ h2
    g["b3"] = np.array([dy.sum()])
    d2 = (dy[:, None] * d["W3"][None, :]) * (1.0 - h2 ** 2)  # dL/d(W2 h1 + b2)
    g["W2"] = (d2.T @ h1).reshape(-1)
    g["b2"] = d2.sum(0)
    d1 = (d2 @ d["W2"]) * (1.0 - h1 ** 2)                  # dL/d(W1 xn + b1)
    g["W1"] = (d1.T @ xn).reshape(-1)
    g["b1"] = d1.sum(0)
    return pack(g)


def init(x, seed=0):
    """Normalisation from the data; weights with variance 1/fan_in, zero biases."""
    rng = np.random.default_rng(seed)
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean(0)
    sd = x.std(0)
    sd = np.where(sd > 1e-6, sd, 1.0)
    return pack({"mu": mu, "sd": sd,
                 "W1": rng.standard_normal((N_H, N_IN)) / np.sqrt(N_IN), "b1": np.zeros(N_H),
                 "W2": rng.standard_normal((N_H, N_H)) / np.sqrt(N_H), "b2": np.zeros(N_H),
                 "W3": rng.standard_normal(N_H) / np.sqrt(N_H), "b3": np.zeros(1)})


# ---------------------------------------------------------------- training (Adam)
# Adam (Kingma & Ba, "Adam: a method for stochastic optimization", 2015, Algorithm 1) with the
# constants the predictor is trained with.  Only the weights and biases are trained: the input
# normalisation mu, sd (the first 32 entries of the parameter vector) stays fixed.
ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8
N_FIXED = 2 * N_IN


def adam_step(p, g, m, v, step, lr):
    """One Adam update of the trainable entries p[N_FIXED:] for gradient g at step number
    ``step`` (1 for the first update).  Returns new (p, m, v); the inputs are not modified.

      m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2
      p <- p - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
    """
    p = np.array(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = ADAM_BETA1 * np.asarray(m, dtype=np.float64) + (1.0 - ADAM_BETA1) * g
    v = ADAM_BETA2 * np.asarray(v, dtype=np.float64) + (1.0 - ADAM_BETA2) * g * g
    mhat = m / (1.0 - ADAM_BETA1 ** step)
    vhat = v / (1.0 - ADAM_BETA2 ** step)
    p[N_FIXED:] -= lr * mhat[N_FIXED:] / (np.sqrt(vhat[N_FIXED:]) + ADAM_EPS)
    return p, m, v


def train(p, x, t, tau, steps, lr):
    """Full-batch Adam on the mean pinball loss (the summed loss of ``loss`` divided by the
    sample count), starting from zero moments.  Returns the final parameters and the mean loss
    before each step."""
    n = len(t)
    p = np.array(p, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    hist = []
    for it in range(1, steps + 1):
        hist.append(loss(p, x, t, tau) / n)
        p, m, v = adam_step(p, grad(p, x, t, tau) / n, m, v, it, lr)
    return p, np.array(hist)
