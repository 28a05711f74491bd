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


def test_adam_update_closed_forms():
    # first step: bias correction gives m_hat = g, v_hat = g^2, so each
    # parameter moves by lr * g / (|g| + eps), about lr against the gradient
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, 1.0, 1.0])
    z = np.zeros(4)
    p, m, v = mlp.adam_update(p0, z, z, g, 1, 0.01)
    assert np.allclose(m, 0.1 * g, rtol=1e-15, atol=0) and np.allclose(v, 0.001 * g * g)
    assert np.allclose(p, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=0)
    # second step with the same gradient: m = 0.19 g, v = 0.001999 g^2,
    # m_hat = 0.19 g / 0.19 = g, v_hat = g^2 again: another step of the same size
    p2, m2, v2 = mlp.adam_update(p, m, v, g, 2, 0.01)
    assert np.allclose(m2, 0.19 * g) and np.allclose(v2, 0.001999 * g * g)
    assert np.allclose(p2 - p, p - p0, rtol=1e-12, atol=1e-15)
    # a gradient that flips sign: m_hat = (0.09 g - 0.1 g) / 0.19 = -g / 19
    p3, m3, v3 = mlp.adam_update(p, m, v, -g, 2, 0.01)
    mh = m3 / (1 - 0.9 ** 2)
    assert np.allclose(mh, -g / 19.0, atol=1e-15)


def test_adam_step_descends():
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (256, mlp.NIN))
    t = mlp.forward(mlp.init(9), X)[0]
    p = mlp.init(10)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for step in range(1, 40):
        p, m, v, lo = mlp.adam_step(p, m, v, step, X, t, 1e-2)
        losses.append(lo)
    assert losses[-1] < 0.5 * losses[0]
