"""Pins of the reference cost-model MLP (float64): central finite differences,
closed forms of degenerate networks, the affine regime, and Adam's first step."""
import numpy as np

from oracle import mlp


def _rand(seed, n=8):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.4, mlp.N_PARAMS)
    X = rng.normal(0.0, 1.0, (n, mlp.F))
    T = rng.normal(0.0, 1.0, n)
    return p, X, T


def test_gradient_matches_central_differences():
    p, X, T = _rand(1)
    g = mlp.grad(p, X, T)
    h = 1e-6
    rng = np.random.default_rng(2)
    # every bias and output weight, and a random sample of the two matrices
    idx = set(rng.choice(mlp.H * mlp.F, 200, replace=False).tolist())
    o = mlp.H * mlp.F
    idx |= set(range(o, o + mlp.H))
    idx |= set((o + mlp.H + rng.choice(mlp.H * mlp.H, 300, replace=False)).tolist())
    idx |= set(range(mlp.N_PARAMS - 2 * mlp.H - 1, mlp.N_PARAMS))
    for i in sorted(idx):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss(pp, X, T) - mlp.loss(pm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_constant_network():
    """All weights zero: y = b3, dL/db3 = 2 mean(b3 - t), every other
    gradient vanishes (hidden units are at the ReLU kink with zero output)."""
    _, X, T = _rand(3)
    p = np.zeros(mlp.N_PARAMS)
    p[-1] = 0.75
    y, _ = mlp.forward(p, X)
    assert np.all(y == 0.75)
    g = mlp.grad(p, X, T)
    assert np.isclose(g[-1], 2.0 * np.mean(0.75 - T), rtol=1e-14, atol=0)
    assert np.all(g[:-1] == 0.0)


def test_single_path_is_a_ramp():
    """One path x_f -> h1[2] -> h2[5] -> y with unit weights: y = max(x_f, 0) * c + b3."""
    _, X, _ = _rand(4, n=64)
    W1 = np.zeros((mlp.H, mlp.F)); W1[2, 7] = 1.0
    W2 = np.zeros((mlp.H, mlp.H)); W2[5, 2] = 1.0
    w3 = np.zeros(mlp.H); w3[5] = -2.5
    p = mlp.pack(W1, np.zeros(mlp.H), W2, np.zeros(mlp.H), w3, 0.125)
    y, _ = mlp.forward(p, X)
    assert np.array_equal(y, np.where(X[:, 7] > 0, X[:, 7], 0.0) * -2.5 + 0.125)


def test_affine_regime_equals_composed_map():
    """Positive weights and inputs keep every unit active: the network is the
    affine map x -> w3^T W2 W1 x + w3^T (W2 b1 + b2) + b3 (non-symmetric W2,
    so a transposed operand fails)."""
    rng = np.random.default_rng(5)
    W1 = rng.uniform(0.1, 1.0, (mlp.H, mlp.F))
    W2 = rng.uniform(0.1, 1.0, (mlp.H, mlp.H))
    b1, b2 = rng.uniform(0, 1, mlp.H), rng.uniform(0, 1, mlp.H)
    w3 = rng.normal(0, 1, mlp.H)
    p = mlp.pack(W1, b1, W2, b2, w3, -0.5)
    X = rng.uniform(0, 1, (32, mlp.F))
    y, _ = mlp.forward(p, X)
    lin = (w3 @ W2) @ W1
    c = w3 @ (W2 @ b1 + b2) - 0.5
    assert np.allclose(y, X @ lin + c, rtol=1e-12, atol=1e-9)
    # and its gradient w.r.t. the input-layer weights is the outer product
    T = np.zeros(32)
    g = mlp.grad(p, X, T)
    dy = 2.0 * (y - T) / 32
    gW1 = g[:mlp.H * mlp.F].reshape(mlp.H, mlp.F)
    assert np.allclose(gW1, np.outer(w3 @ W2, dy @ X), rtol=1e-10, atol=1e-12)


def test_adam_first_step_is_signed_learning_rate():
    """With zero moments, the bias-corrected first step is -lr * g / |g|
    (eps -> 0), whatever the gradient's magnitude."""
    g = np.array([3.0, -1e-3, 250.0, -7.0])
    p, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)


def test_adam_fits_a_linear_target():
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (128, mlp.F))
    T = 0.5 * X[:, 0] - X[:, 3] + 2.0
    p = rng.normal(0, 0.1, mlp.N_PARAMS)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0 = mlp.loss(p, X, T)
    for step in range(1, 301):
        p, m, v = mlp.adam(p, mlp.grad(p, X, T), m, v, step, lr=3e-3)
    assert mlp.loss(p, X, T) < 0.02 * l0
