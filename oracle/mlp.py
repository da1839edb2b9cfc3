"""FP64 reference of the learned smoothing-parameter network (oracle, test
infrastructure).

The damping eta of the additive Schwarz smoother (equation ASM, eta in (0,1))
and the number of smoothing steps of Algorithm 1 are predicted per smoothed
level by a small multilayer perceptron:

    x = (log10(nu) / 2, log10(sigma) / 4, |a| h / nu, k - 1.5)
    h1 = tanh(W1 x + b1)          (32)
    h2 = tanh(W2 h1 + b2)         (32)
    z  = W3 h2 + b3               (10 outputs)
    eta_l = 1 / (1 + exp(-z_l))              outputs 0..4, finest level first
    steps_l = clamp(round(z_{5+l}), 1, 8)    outputs 5..9, finest level first

Training loss: masked mean squared error (weights M) of the outputs against
the sweep's targets (logits of the best dampings, best step counts).
Parameters are packed as [W1 (32x4, row-major), b1, W2 (32x32), b2,
W3 (10x32), b3].
"""
import numpy as np

NIN, H, NOUT = 4, 32, 10
NETA = 5          # damping outputs; the step-count outputs follow
SHAPES = [("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (NOUT, H)), ("b3", (NOUT,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def features(nu, sigma, amag, N, k):
    """Input features of one problem: amag = max|a|, h = 1/N."""
    return np.array([np.log10(nu) / 2.0, np.log10(sigma) / 4.0, amag / (N * nu), k - 1.5])


def forward(theta, X):
    """Logits (n, NOUT) for features X (n, NIN)."""
    p = unpack(theta)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    return h2 @ p["W3"].T + p["b3"]


def steps(z):
    """Smoothing steps from the count outputs (round half away from zero,
    clamped to [1, 8])."""
    return np.clip(np.sign(z) * np.floor(np.abs(z) + 0.5), 1, 8).astype(int)


def loss(theta, X, Y, M):
    """Masked mean squared error of the outputs."""
    Z = forward(theta, X)
    return float(np.sum(M * (Z - Y) ** 2) / np.sum(M))


def grad(theta, X, Y, M):
    """Gradient of `loss` by the chain rule through both tanh layers."""
    p = unpack(theta)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    Z = h2 @ p["W3"].T + p["b3"]
    dZ = 2.0 * M * (Z - Y) / np.sum(M)
    g = {"W3": dZ.T @ h2, "b3": dZ.sum(axis=0)}
    d2 = (dZ @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])


def init(seed):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)


def adam_step(theta, g, m, v, t, lr=1e-2, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
