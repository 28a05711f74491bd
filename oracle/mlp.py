"""fp64 reference of the linking-length proposer network (TEST INFRASTRUCTURE).

24 -> 64 -> 64 -> 1 with ReLU, loss mean((y - t)^2); parameters flattened as
W1[64][24], b1[64], W2[64][64], b2[64], W3[64], b3.  Forward and backward
are written out layer by layer in numpy float64; the tests pin them with
central finite differences.
"""
import numpy as np

NIN, NH = 24, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)),
         ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unflatten(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def forward(p, X):
    w = unflatten(p)
    X = np.asarray(X, np.float64)
    a1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w["W3"] + w["b3"][0]
    return y, (X, a1, h1, a2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p, X, t):
    w = unflatten(p)
    y, (X, a1, h1, a2, h2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, np.float64)) / n
    g = {"W3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dy, w["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ w["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return np.concatenate([g[name].ravel() for name, _ in SIZES])


def init(seed=0):
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) > 1 else NH
            parts.append(rng.normal(0, np.sqrt(2.0 / fan_in), shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts)


def adam_update(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) in fp64: moments
    m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, bias-corrected
    m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t), then
    p <- p - lr m_hat / (sqrt(v_hat) + eps).  Returns new (p, m, v)."""
    p, m, v, g = (np.asarray(a, np.float64) for a in (p, m, v, g))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def adam_step(p, m, v, step, X, t, lr):
    """One training step: the loss before the update, then Adam on the
    minibatch gradient.  Returns (p, m, v, loss)."""
    lo = loss(p, X, t)
    p, m, v = adam_update(p, m, v, grad(p, X, t), step, lr)
    return p, m, v, lo
