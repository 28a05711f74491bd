"""Pins for the fp64 proposer-network reference (CPU): central finite
differences of the loss match its analytic gradient; a zero hidden layer
gives the closed-form gradient of a constant predictor."""
import numpy as np

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init(1) + rng.normal(0, 0.05, mlp.NPARAM)
    X = rng.normal(0, 1, (40, mlp.NIN))
    t = rng.normal(0, 1, 40)
    g = mlp.grad(p, X, t)
    idx = rng.choice(mlp.NPARAM, 300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM); e[i] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_constant_predictor_closed_form():
    # all weights zero, output bias b: y = b everywhere; dL/db = 2 mean(b - t),
    # every other gradient is zero (ReLU of zero pre-activations)
    p = np.zeros(mlp.NPARAM); p[-1] = 0.75
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (17, mlp.NIN)); t = rng.normal(0, 1, 17)
    g = mlp.grad(p, X, t)
    assert np.isclose(g[-1], 2 * np.mean(0.75 - t))
    assert np.all(g[:-1] == 0)


def test_descent_direction_lowers_loss():
    rng = np.random.default_rng(2)
    p = mlp.init(3)
    X = rng.normal(0, 1, (64, mlp.NIN)); t = rng.normal(0, 1, 64)
    g = mlp.grad(p, X, t)
    assert mlp.loss(p - 1e-3 * g, X, t) < mlp.loss(p, X, t)
