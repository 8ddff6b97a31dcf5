"""Per-orbital MLP of the learned fsGW warm start, oracle side (FP64 NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The warm start is not in the paper; the model follows this reading:
  * features per orbital p: eps_p, (L L^T)_pp = sum_{P,q} L[P,p,q]^2, and
    eps_p - mu_mid with mu_mid = (eps_HOMO + eps_LUMO) / 2;
  * inputs standardised with a fixed mean / std (from the training set),
    targets delta_p = F*_pp - eps_p standardised the same way;
  * network 3 -> 128 -> 128 -> 128 -> 1 with SiLU, x * sigmoid(x), after each
    hidden layer; loss the mean squared error of the standardised output;
  * Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction.
Parameters are one flat vector in the order W1 [128][3], b1, W2 [128][128],
b2, W3 [128][128], b3, W4 [1][128], b4.
"""
from __future__ import annotations

import numpy as np

SIZES = (3, 128, 128, 128, 1)


def param_count(sizes=SIZES):
    return sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1))


def unpack(theta, sizes=SIZES):
    """Flat vector -> [(W, b), ...] views."""
    out, o = [], 0
    for i in range(len(sizes) - 1):
        n_in, n_out = sizes[i], sizes[i + 1]
        W = theta[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = theta[o:o + n_out]
        o += n_out
        out.append((W, b))
    return out


def features(eps, L, nocc):
    """[nmo][3]: eps_p, (L L^T)_pp, eps_p - mu_mid."""
    eps = np.asarray(eps, dtype=float)
    llt = np.einsum("Ppq,Ppq->p", L, L)
    mu = 0.5 * (eps[nocc - 1] + eps[nocc])
    return np.stack([eps, llt, eps - mu], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, norm):
    """norm = (mean_x[3], std_x[3], mean_t, std_t).  Returns (y, cache) with
    y in target units."""
    mx, sx, mt, st = norm
    a = (np.asarray(X, dtype=float) - mx) / sx
    cache = [a]
    layers = unpack(theta)
    for i, (W, b) in enumerate(layers):
        z = a @ W.T + b
        if i < len(layers) - 1:
            cache.append(z)
            a = silu(z)
            cache.append(a)
        else:
            out = z[:, 0]
    return mt + st * out, cache


def loss(theta, X, T, norm):
    y, _ = forward(theta, X, norm)
    st = norm[3]
    return float(np.mean(((y - T) / st) ** 2))


def backward(theta, X, T, norm):
    """Gradient of the loss with respect to the flat parameters."""
    mx, sx, mt, st = norm
    y, cache = forward(theta, X, norm)
    B = X.shape[0]
    layers = unpack(theta)
    grads = []
    d = (2.0 / B) * ((y - T) / st)[:, None]          # dL / d(standardised output)
    nl = len(layers)
    for i in range(nl - 1, -1, -1):
        W, b = layers[i]
        a_in = cache[0] if i == 0 else cache[2 * i]
        grads.append((d.T @ a_in, d.sum(axis=0)))
        if i > 0:
            z_prev = cache[2 * i - 1]
            d = (d @ W) * dsilu(z_prev)
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db.ravel())
    return np.concatenate(flat)


def adam_step(theta, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
