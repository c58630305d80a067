"""Pins of the FP64 MLP reference: finite differences, a hand-computed network, Adam's first step."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    in_dim, H, B = 5, 7, 11
    p = rng.normal(scale=0.5, size=mlp.n_params(in_dim, H))
    X = rng.normal(size=(B, in_dim))
    T = rng.normal(size=B)
    loss, g = mlp.loss_grad(X, T, p, in_dim, H)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(p.size):
        a, b = p.copy(), p.copy()
        a[i] += h
        b[i] -= h
        num[i] = (mlp.loss_grad(X, T, a, in_dim, H)[0] - mlp.loss_grad(X, T, b, in_dim, H)[0]) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-8)


def test_hand_computed_network():
    # in = 1, H = 2: W1 = [1, -1], b1 = [0, 1], W2 = [[2, 0], [1, 1]], b2 = [0, -1], w3 = [1, 3], b3 = 0.5
    p = np.array([1.0, -1.0, 0.0, 1.0, 2.0, 0.0, 1.0, 1.0, 0.0, -1.0, 1.0, 3.0, 0.5])
    # x = 2: z1 = [2, -1] -> h1 = [2, 0]; z2 = [4, 0 - 1] -> h2 = [4, 0]; y = 4 + 0.5
    y, _ = mlp.forward(np.array([[2.0]]), p, 1, 2)
    assert y[0] == 4.5
    # loss against t = 4: (0.5)^2; dL/db3 = 2 * 0.5 = 1; dL/dw3 = h2 = [4, 0]
    loss, g = mlp.loss_grad(np.array([[2.0]]), np.array([4.0]), p, 1, 2)
    assert loss == 0.25
    assert g[-1] == 1.0
    np.testing.assert_array_equal(g[-3:-1], [4.0, 0.0])


def test_adam_first_step_moves_by_lr():
    # after bias correction the first Adam step is lr * g / (|g| + eps) ~ lr * sign(g)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    q, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-12, 1)
    np.testing.assert_allclose(q, p - 0.01 * np.sign(g), rtol=0, atol=1e-9)
