"""Pins of the float64 policy-network reference (oracle/mlp.py).

Each check ties the reference to something other than itself: central finite
differences of the loss, the closed form of the network when every hidden
unit is active (a linear model), the all-dead case (a constant), Adam's
first step in closed form, and a teacher network that training must recover.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def rand_params(rng, scale=0.5):
    return rng.normal(0.0, scale, mlp.NPARAM)


def test_layout():
    assert mlp.NPARAM == 513
    p = np.arange(mlp.NPARAM, dtype=np.float64)
    W1, b1, w2, b2 = mlp.unpack(p)
    assert W1[0, 0] == 0 and W1[1, 0] == 6 and W1[63, 5] == 383
    assert b1[0] == 384 and w2[0] == 448 and b2 == 512
    assert np.array_equal(mlp.pack(W1, b1, w2, b2), p)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = rand_params(rng)
    X = rng.normal(0, 1, (37, 6))
    t = rng.normal(0, 1, 37)
    _, g = mlp.loss_and_grad(p, X, t)
    h = 1e-6
    # away from ReLU kinks: skip coordinates whose perturbation flips a unit
    _, z = mlp.forward(p, X)
    assert np.min(np.abs(z)) > 1e-4
    num = np.empty_like(p)
    for k in range(mlp.NPARAM):
        e = np.zeros_like(p)
        e[k] = h
        num[k] = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_all_units_active_is_a_linear_model():
    rng = np.random.default_rng(2)
    W1 = rng.normal(0, 0.1, (64, 6))
    b1 = np.full(64, 50.0)  # every pre-activation positive on these inputs
    w2 = rng.normal(0, 1, 64)
    b2 = 0.3
    p = mlp.pack(W1, b1, w2, b2)
    X = rng.normal(0, 1, (20, 6))
    t = rng.normal(0, 1, 20)
    # y = a . x + c with a = W1^T w2, c = w2 . b1 + b2
    a = W1.T @ w2
    c = w2 @ b1 + b2
    y, _ = mlp.forward(p, X)
    assert np.allclose(y, X @ a + c, rtol=0, atol=1e-9)
    L, g = mlp.loss_and_grad(p, X, t)
    r = X @ a + c - t
    assert math.isclose(L, float(np.mean(r ** 2)), rel_tol=1e-12)
    dy = 2 * r / len(t)
    gW1, gb1, gw2, gb2 = mlp.unpack(g)
    assert np.allclose(gW1, np.outer(w2, X.T @ dy), atol=1e-9)
    assert np.allclose(gb1, w2 * dy.sum(), atol=1e-9)
    assert np.allclose(gw2, (X @ W1.T + b1).T @ dy, atol=1e-9)
    assert math.isclose(gb2, dy.sum(), rel_tol=1e-12, abs_tol=1e-12)


def test_dead_units_give_a_constant():
    rng = np.random.default_rng(3)
    W1 = rng.normal(0, 0.01, (64, 6))
    b1 = np.full(64, -10.0)
    p = mlp.pack(W1, b1, rng.normal(0, 1, 64), -0.7)
    X = rng.normal(0, 1, (15, 6))
    t = rng.normal(0, 1, 15)
    y, _ = mlp.forward(p, X)
    assert np.allclose(y, -0.7)
    L, g = mlp.loss_and_grad(p, X, t)
    gW1, gb1, gw2, gb2 = mlp.unpack(g)
    assert not gW1.any() and not gb1.any() and not gw2.any()
    assert math.isclose(gb2, 2 * np.mean(-0.7 - t), rel_tol=1e-12)
    assert math.isclose(L, np.mean((-0.7 - t) ** 2), rel_tol=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rand_params(rng)
    g = rng.normal(0, 1, mlp.NPARAM)
    lr, eps = 1e-2, 1e-8
    p1, m, v = mlp.adam_step(p, np.zeros_like(p), np.zeros_like(p), g, 1, lr, eps=eps)
    # bias-corrected moments equal g and g^2 on the first step
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_recovers_a_teacher():
    rng = np.random.default_rng(5)
    teacher = rand_params(rng, 0.4)
    X = rng.normal(0, 1, (256, 6))
    t, _ = mlp.forward(teacher, X)
    p = rand_params(np.random.default_rng(6), 0.4)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss_and_grad(p, X, t)[0]
    for s in range(1, 1501):
        L, g = mlp.loss_and_grad(p, X, t)
        p, m, v = mlp.adam_step(p, m, v, g, s, 3e-3)
    assert L < 0.02 * L0


def test_policy_eps_clamps_and_falls_back():
    p = np.zeros(mlp.NPARAM)
    x = mlp.features(1000, 50, 0, 0, 0, 0, 0.5, 0)
    p[-1] = math.log(2.0)
    assert math.isclose(mlp.policy_eps(p, x, 1 / 16, 16), 2.0, rel_tol=1e-12)
    p[-1] = 10.0
    assert mlp.policy_eps(p, x, 1 / 16, 16) == 16
    p[-1] = -10.0
    assert mlp.policy_eps(p, x, 1 / 16, 16) == 1 / 16
    p[-1] = float("nan")
    assert mlp.policy_eps(p, x, 1 / 16, 16) is None


def test_features():
    x = mlp.features(1000, 0, 5, 10, 30, 2000, 0.5, 3)
    assert np.allclose(x, [math.log(1000), 0.0, 0.5, 0.015, 0.5, 3.0])
    x0 = mlp.features(1000, 7, 0, 0, 0, 0, 0.25, 0)
    assert np.allclose(x0, [math.log(1000), math.log(7), 0, 0, 0.25, 0])


@pytest.mark.parametrize("n", [0, 1])
def test_tiny_batches(n):
    rng = np.random.default_rng(7)
    p = rand_params(rng)
    X = rng.normal(0, 1, (n, 6))
    t = rng.normal(0, 1, n)
    L, g = mlp.loss_and_grad(p, X, t)
    if n == 0:
        assert L == 0.0 and not g.any()
    else:
        assert np.isfinite(g).all()


def test_committed_policy_weights():
    """The trained policy file loads, has 513 finite weights and a clamp range
    inside the library's eps limits; its outputs on typical features are finite."""
    from paper_1507_05086_amd import policy
    w, lo, hi = policy.load()
    assert w.shape == (mlp.NPARAM,) and np.isfinite(w).all()
    assert 0 < lo <= hi <= 1000
    for x in ([math.log(6.7e7), math.log(2e5), 0, 0, 0.5, 0], [math.log(1e5), math.log(30), 0.1, 0.3, 4.0, 120]):
        e = mlp.policy_eps(w.astype(np.float64), np.array(x), lo, hi)
        assert e is not None and lo <= e <= hi
