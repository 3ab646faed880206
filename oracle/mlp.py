"""Reference for the learned contraction-order cost model (test infrastructure
only: tests, the smoke check and the benchmark's CPU leg use it; the library
never does).

A multilayer perceptron F -> H -> H -> 1 with ReLU hidden units, in float64,
written from the textbook definitions: affine maps and max(0, .), the mean
squared error L = (1/n) sum_s (y_s - t_s)^2, its gradient by the chain rule,
and the Adam update (Kingma and Ba, 2015, Algorithm 1, with bias correction).

Flat parameter layout (the interface shared with the GPU model):
    W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3
"""
import numpy as np

F = 16
H = 64
N_PARAMS = H * F + H + H * H + H + H + 1


def unpack(p):
    """Views of the flat parameter vector as (W1, b1, W2, b2, w3, b3)."""
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,), p.shape
    o = 0
    W1 = p[o:o + H * F].reshape(H, F)
    o += H * F
    b1 = p[o:o + H]
    o += H
    W2 = p[o:o + H * H].reshape(H, H)
    o += H * H
    b2 = p[o:o + H]
    o += H
    w3 = p[o:o + H]
    o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(w3),
                           np.atleast_1d(b3)]).astype(np.float64)


def forward(p, X):
    """Predictions y[n] for inputs X[n][F]; also the pre-activations."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, a1, h1, a2, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    d = y - np.asarray(T, dtype=np.float64)
    return float(np.mean(d * d))


def grad(p, X, T):
    """dL/dp for the mean squared error, by backpropagation."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (X, a1, h1, a2, h2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(T, dtype=np.float64)) / n          # dL/dy
    gw3 = h2.T @ dy
    gb3 = dy.sum()
    da2 = np.outer(dy, w3) * (a2 > 0.0)                             # dL/da2
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0.0)                                   # dL/da1
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gw3, gb3)


def adam(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
