"""Pins of the cost-model oracle: the backpropagated gradient equals central finite
differences of the loss, and structural special cases hold."""
import numpy as np

import oracle.mlp as M

RNG = np.random.default_rng(3)


def rand_params(scale=0.5):
    return RNG.normal(0, scale, M.N_PARAMS)


def test_parameter_count():
    assert M.N_PARAMS == 7 * 64 + 64 + 64 * 64 + 64 + 64 + 1


def test_gradient_matches_finite_differences():
    p = rand_params()
    X = RNG.normal(0, 1, (9, 7))
    y = RNG.normal(0, 1, 9)
    g = M.grad(p, X, y)
    h = 1e-6
    idx = RNG.choice(M.N_PARAMS, 300, replace=False)
    idx = np.concatenate([idx, [M.N_PARAMS - 1, 0, 7 * 64, 7 * 64 + 64 + 64 * 64 + 64]])  # b3, W1, b1, w3 first
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        fd = (M.loss(p + e, X, y) - M.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_linear_region_reduces_to_least_squares_gradient():
    """with every unit active and W2 = I, w3 = 1: f(x) = sum(W1^T x + b1) + b2 sum + b3,
    and d loss / d b3 = 2 mean(f - y)"""
    q = {"W1": np.abs(RNG.normal(0, 1, (7, 64))), "b1": np.ones(64), "W2": np.eye(64), "b2": np.zeros(64),
         "w3": np.ones(64), "b3": np.array([0.3])}
    p = M.pack(q)
    X = np.abs(RNG.normal(0, 1, (5, 7)))
    y = RNG.normal(0, 1, 5)
    f = (X @ q["W1"] + 1.0).sum(axis=1) + 0.3
    out, _ = M.forward(p, X)
    assert np.allclose(out, f)
    assert np.isclose(M.grad(p, X, y)[-1], 2 * np.mean(f - y))


def test_dead_units_have_zero_gradient():
    q = M.unpack(rand_params())
    q["b1"][:] = -1e6  # every first-layer unit off: output = w3 . relu(b2) + b3
    p = M.pack(q)
    X = RNG.normal(0, 1, (4, 7))
    g = M.unpack(M.grad(p, X, RNG.normal(0, 1, 4)))
    assert np.all(g["W1"] == 0) and np.all(g["b1"] == 0) and np.all(g["W2"] == 0)
