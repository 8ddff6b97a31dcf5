"""Pins of the warm-start MLP oracle: central finite differences of the loss,
closed forms of the network at special parameters, the SiLU derivative, and
the first Adam step (bias correction makes it lr * sign(g))."""
import numpy as np

import gwsynth
from oracle import mlp


def _setup(seed=0, B=9):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.param_count()) * 0.2
    X = rng.standard_normal((B, 3)) * np.array([1.0, 0.1, 0.5]) + np.array([0.2, 0.05, 0.0])
    T = rng.standard_normal(B) * 1e-3
    norm = (np.array([0.1, 0.04, 0.0]), np.array([0.9, 0.08, 0.6]), 2e-4, 1.5e-3)
    return theta, X, T, norm


def test_parameter_count():
    assert mlp.param_count() == 3 * 128 + 128 + 2 * (128 * 128 + 128) + 128 + 1 == 33665


def test_gradient_matches_central_differences():
    theta, X, T, norm = _setup()
    g = mlp.backward(theta, X, T, norm)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(mlp.param_count(), 40, replace=False),
                          [0, 384, 512, 16640, 33536, 33664]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T, norm) - mlp.loss(tm, X, T, norm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_weights_give_the_output_bias():
    theta, X, T, norm = _setup()
    layers = mlp.unpack(theta)
    for W, b in layers:
        W[...] = 0.0
    layers[-1][1][0] = 0.7
    y, _ = mlp.forward(theta, X, norm)
    # hidden activations are silu(b), the last layer ignores them (W4 = 0)
    assert np.allclose(y, norm[2] + norm[3] * 0.7, rtol=0, atol=1e-15)


def test_linear_regime_matches_the_product_of_layers():
    """Tiny weights: silu(z) = z/2 + z^2/4 + O(z^4), so with zero biases the
    network is (1/8) W4 W3 W2 W1 x up to a relative O(|z|) ~ 1e-4 correction."""
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(mlp.param_count()) * 1e-4
    layers = mlp.unpack(theta)
    for _, b in layers:
        b[...] = 0.0
    norm = (np.zeros(3), np.ones(3), 0.0, 1.0)
    X = rng.standard_normal((4, 3))
    y, _ = mlp.forward(theta, X, norm)
    W1, W2, W3, W4 = (l[0] for l in layers)
    lin = (X @ W1.T @ W2.T @ W3.T @ W4.T)[:, 0] / 8.0
    assert np.abs(y - lin).max() < 1e-3 * np.abs(lin).max()


def test_silu_derivative():
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.dsilu(z)).max() < 1e-9


def test_first_adam_step_is_lr_times_sign():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(theta - new, 1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-15)


def test_features():
    o, v, A = 3, 7, 12
    eps, L = gwsynth.system(o, v, A, 4)
    f = mlp.features(eps, L, o)
    p = 4
    assert f[p, 0] == eps[p]
    assert abs(f[p, 1] - sum(L[P, p, q] ** 2 for P in range(A) for q in range(o + v))) < 1e-14
    assert abs(f[p, 2] - (eps[p] - 0.5 * (eps[o - 1] + eps[o]))) < 1e-15
