"""Plain FP64 reference of the warm-start network (test infrastructure only).

The network: hidden layers h_l = tanh(W_l h_{l-1} + b_l), l = 1..L, a linear
output y = W_{L+1} h_L + b_{L+1} of n_comb groups of n_out values, and the
prediction pred[o] = sum_r c[r] y[r n_out + o] with the row's coefficients c.
Loss: mean over rows and outputs of (pred - target)^2.  Parameters: per layer
the row-major matrix [W_l b_l] (bias in the last column), layers in order.

The gradient is the chain rule written out layer by layer (backpropagation);
the tests pin it against central finite differences.  The optimiser is Adam
as defined by Kingma & Ba (2015, Algorithm 1), with the bias-corrected
moments written out as in that algorithm.
"""
from __future__ import annotations

import numpy as np


def dims(n_in, n_hidden, n_layers, n_comb, n_out):
    return [n_in] + [n_hidden] * n_layers + [n_comb * n_out]


def unpack(theta, d):
    """Per layer (W, b) views of the flat parameter vector."""
    out, off = [], 0
    for a, b in zip(d[:-1], d[1:]):
        Wb = np.asarray(theta[off:off + b * (a + 1)], dtype=np.float64).reshape(b, a + 1)
        out.append((Wb[:, :a], Wb[:, a]))
        off += b * (a + 1)
    if off != len(theta):
        raise ValueError("parameter count does not match the architecture")
    return out


def forward(arch, theta, X, Cc):
    """Hidden activations, raw output y and prediction for rows X [n, n_in]."""
    n_in, n_hidden, n_layers, n_comb, n_out = arch
    layers = unpack(theta, dims(*arch))
    h = [np.asarray(X, dtype=np.float64)]
    for W, b in layers[:-1]:
        h.append(np.tanh(h[-1] @ W.T + b))
    W, b = layers[-1]
    y = h[-1] @ W.T + b
    Cc = np.asarray(Cc, dtype=np.float64)
    pred = np.zeros((X.shape[0], n_out))
    for r in range(n_comb):
        pred += Cc[:, r:r + 1] * y[:, r * n_out:(r + 1) * n_out]
    return h, y, pred


def loss(arch, theta, X, Cc, T):
    _, _, pred = forward(arch, theta, X, Cc)
    return float(np.mean((pred - np.asarray(T, dtype=np.float64)) ** 2))


def grad(arch, theta, X, Cc, T):
    """d loss / d theta by backpropagation."""
    n_in, n_hidden, n_layers, n_comb, n_out = arch
    d = dims(*arch)
    layers = unpack(theta, d)
    h, y, pred = forward(arch, theta, X, Cc)
    n = X.shape[0]
    dpred = 2.0 * (pred - np.asarray(T, dtype=np.float64)) / (n * n_out)
    Cc = np.asarray(Cc, dtype=np.float64)
    dz = np.zeros_like(y)
    for r in range(n_comb):
        dz[:, r * n_out:(r + 1) * n_out] = Cc[:, r:r + 1] * dpred
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = np.concatenate([dz.T @ h[l], dz.sum(axis=0)[:, None]], axis=1)
        if l > 0:
            dh = dz @ W
            dz = dh * (1.0 - h[l] ** 2)
    return np.concatenate([g.ravel() for g in grads])


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
