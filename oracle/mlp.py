"""Float64 reference of the epsilon-policy network.

TEST INFRASTRUCTURE ONLY (see the package docstring): the GPU training and
inference kernels are checked against these functions; the library never
imports them.

The network replaces the fixed rule of Algorithm 2 (B_i = ceil(eps n_i /
Delta_i)) by a per-round eps_i; the paper itself uses one fixed eps, so the
network, its features and its training are additions of this project:

  x_i   = [ln n_i, ln max(Delta_i, 1), conflicts_{i-1} / B_{i-1},
           claimed_{i-1} / n_{i-1}, eps_{i-1}, i]        (zeros and the call's
                                                         eps in round 0)
  z     = W1 x + b1            W1: 64 x 6, b1: 64
  h     = relu(z)              (derivative 0 at z <= 0)
  y     = w2 . h + b2          w2: 64, b2: scalar
  eps_i = clamp(exp(y), eps_min, eps_max); a non-finite y falls back to the
          fixed rule.

Parameters are one float vector laid out W1 (row-major), b1, w2, b2 (513
values).  Training minimises the mean squared error L = mean((y - t)^2)
against targets t = ln eps* with Adam.
"""
from __future__ import annotations

import math

import numpy as np

IN, HID = 6, 64
NPARAM = HID * IN + HID + HID + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAM,)
    W1 = p[: HID * IN].reshape(HID, IN)
    b1 = p[HID * IN: HID * IN + HID]
    w2 = p[HID * IN + HID: HID * IN + 2 * HID]
    b2 = p[HID * IN + 2 * HID]
    return W1, b1, w2, b2


def pack(W1, b1, w2, b2):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(w2), [float(b2)]]).astype(np.float64)


def forward(p, X):
    """y[N] for inputs X[N, 6]; also returns the pre-activations z[N, 64]."""
    W1, b1, w2, b2 = unpack(p)
    X = np.asarray(X, dtype=np.float64).reshape(-1, IN)
    z = X @ W1.T + b1
    h = np.maximum(z, 0.0)
    return h @ w2 + b2, z


def loss_and_grad(p, X, t):
    """L = mean((y - t)^2) and dL/dp (backpropagation through the two layers)."""
    W1, b1, w2, b2 = unpack(p)
    X = np.asarray(X, dtype=np.float64).reshape(-1, IN)
    t = np.asarray(t, dtype=np.float64).ravel()
    n = len(t)
    y, z = forward(p, X)
    r = y - t
    L = float(np.mean(r * r)) if n else 0.0
    dy = 2.0 * r / n if n else r
    h = np.maximum(z, 0.0)
    g_w2 = h.T @ dy
    g_b2 = float(dy.sum())
    dz = np.outer(dy, w2) * (z > 0.0)
    g_W1 = dz.T @ X
    g_b1 = dz.sum(axis=0)
    return L, pack(g_W1, g_b1, g_w2, g_b2)


def adam_step(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; step >= 1.
    Returns the new (p, m, v)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def features(n_rem, delta, conflicts_prev, b_prev, claimed_prev, n_prev, eps_prev, i):
    """The six per-round inputs of round i (see the module docstring)."""
    if i == 0:
        return np.array([math.log(n_rem), math.log(max(delta, 1)), 0.0, 0.0, eps_prev, 0.0])
    return np.array([math.log(n_rem), math.log(max(delta, 1)),
                     conflicts_prev / b_prev if b_prev > 0 else 0.0,
                     claimed_prev / n_prev if n_prev > 0 else 0.0, eps_prev, float(i)])


def policy_eps(p, x, eps_min, eps_max):
    """eps_i for one feature vector, or None when the output is not finite
    (the caller then keeps the fixed rule)."""
    with np.errstate(all="ignore"):
        y, _ = forward(p, np.asarray(x, np.float64)[None, :])
        y = float(y[0])
        if not math.isfinite(y):
            return None
        e = math.exp(y) if y < 700 else math.inf
    return min(max(e, eps_min), eps_max)
