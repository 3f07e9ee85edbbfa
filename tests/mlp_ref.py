"""Plain fp64 numpy version of the size predictor's perceptron, for checking
the device kernels: y = w2 . relu(W1 x + b1) + b2, loss = mean (y - t)^2 / 2.
Parameter order: W1 [H][F] row-major, b1 [H], w2 [H], b2."""
import numpy as np


def unpack(p, F, H):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[:H * F].reshape(H, F)
    b1 = p[H * F:H * F + H]
    w2 = p[H * F + H:H * F + 2 * H]
    b2 = p[H * F + 2 * H]
    return W1, b1, w2, b2


def forward(p, X, F, H):
    W1, b1, w2, b2 = unpack(p, F, H)
    Z = np.asarray(X, np.float64) @ W1.T + b1
    return np.maximum(Z, 0.0) @ w2 + b2


def loss(p, X, t, F, H):
    e = forward(p, X, F, H) - np.asarray(t, np.float64)
    return 0.5 * np.mean(e * e)


def grad(p, X, t, F, H):
    """Backpropagation by hand."""
    X = np.asarray(X, np.float64)
    W1, b1, w2, b2 = unpack(p, F, H)
    Z = X @ W1.T + b1
    Hh = np.maximum(Z, 0.0)
    y = Hh @ w2 + b2
    dy = (y - np.asarray(t, np.float64)) / X.shape[0]
    dH = np.outer(dy, w2) * (Z > 0)
    return np.concatenate([(dH.T @ X).ravel(), dH.sum(axis=0), Hh.T @ dy, [dy.sum()]])
