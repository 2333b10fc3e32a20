"""Pins of the network oracle: backpropagation against central finite
differences, closed forms of special cases, and Adam's first-step property
(at t = 1 the bias-corrected moments are g and g^2, so every parameter moves
by lr g / (|g| + eps), Kingma & Ba 2015, Section 2.1)."""
import numpy as np

from oracle import nn

ARCH = (5, 7, 2, 3, 4)


def _data(seed=0, n=9):
    rng = np.random.default_rng(seed)
    d = nn.dims(*ARCH)
    theta = rng.standard_normal(sum(b * (a + 1) for a, b in zip(d[:-1], d[1:]))) * 0.5
    X = rng.standard_normal((n, ARCH[0]))
    Cc = rng.uniform(0.5, 1.5, size=(n, ARCH[3]))
    T = rng.standard_normal((n, ARCH[4]))
    return theta, X, Cc, T


def test_backprop_matches_central_differences():
    theta, X, Cc, T = _data()
    g = nn.grad(ARCH, theta, X, Cc, T)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(len(theta)):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (nn.loss(ARCH, theta + e, X, Cc, T) - nn.loss(ARCH, theta - e, X, Cc, T)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_zero_hidden_weights_give_the_closed_form():
    # with W_1 = 0 every row sees h_1 = tanh(b_1); then the output is affine in that constant
    arch = (3, 2, 1, 1, 2)
    b1 = np.array([0.3, -0.7])
    W2 = np.array([[1.0, 2.0], [-1.0, 0.5]])
    b2 = np.array([0.25, -0.5])
    theta = np.concatenate([np.column_stack([np.zeros((2, 3)), b1]).ravel(), np.column_stack([W2, b2]).ravel()])
    X = np.random.default_rng(1).standard_normal((4, 3))
    c = np.array([[1.0], [2.0], [0.5], [-1.0]])
    _, _, pred = nn.forward(arch, theta, X, c)
    base = W2 @ np.tanh(b1) + b2
    np.testing.assert_allclose(pred, c * base[None, :], rtol=1e-15, atol=1e-15)


def test_prediction_is_linear_in_the_coefficients():
    theta, X, Cc, T = _data(2)
    _, _, p1 = nn.forward(ARCH, theta, X, Cc)
    _, _, p2 = nn.forward(ARCH, theta, X, 2.0 * Cc)
    _, _, p3 = nn.forward(ARCH, theta, X, Cc[:, [1, 0, 2]] * np.array([0, 0, 1.0]))
    np.testing.assert_allclose(p2, 2 * p1, rtol=1e-14, atol=1e-14)
    _, y, _ = nn.forward(ARCH, theta, X, Cc)
    np.testing.assert_allclose(p3, Cc[:, 2:3] * y[:, 2 * ARCH[4]:3 * ARCH[4]], rtol=1e-14, atol=1e-14)


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.02, 1e-3, -50.0])
    theta = np.zeros(4)
    th, m, v = nn.adam_step(theta, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_converges_on_a_quadratic():
    theta = np.array([2.0, -3.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 3001):
        g = 2.0 * (theta - np.array([0.5, 1.5]))
        theta, m, v = nn.adam_step(theta, g, m, v, t, lr=0.01)
    np.testing.assert_allclose(theta, [0.5, 1.5], atol=1e-3)
