"""Pins of the FP64 cost-network oracle: a hand-computed forward pass, the
gradient against central finite differences of the loss, and Adam's first
step (whose bias-corrected size is the learning rate)."""
import numpy as np

from oracle import mlp


def test_forward_hand_computed():
    F = 1
    p = np.zeros(mlp.n_params(F))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p.copy(), F)
    # offsets into the flat layout
    o_b1 = 64 * F
    o_w2 = o_b1 + 64
    o_b2 = o_w2 + 64 * 64
    o_w3 = o_b2 + 64
    o_b3 = o_w3 + 64
    p[0] = 2.0          # W1[0][0]
    p[o_b1] = -1.0      # b1[0]
    p[o_w2] = 3.0       # W2[0][0]
    p[o_w3] = 0.5       # W3[0]
    p[o_b3] = 0.25      # b3
    y = mlp.forward(p, np.array([[2.0], [0.0], [0.25]]), F)
    # x=2: relu(2*2-1)=3 -> relu(3*3)=9 -> 0.5*9+0.25 ; x=0 and x=0.25: hidden unit off
    assert y.tolist() == [4.75, 0.25, 0.25]
    assert mlp.loss(p, [[2.0], [0.0]], [4.0, 0.25], F) == (0.75 ** 2) / 2


def test_gradient_matches_central_differences():
    F = 5
    rng = np.random.default_rng(0)
    p = mlp.init(F, seed=1)
    x = rng.normal(size=(37, F))
    t = rng.normal(size=37)
    L, g = mlp.loss_grad(p, x, t, F)
    assert np.isclose(L, mlp.loss(p, x, t, F))
    idx = rng.choice(p.size, 80, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, t, F) - mlp.loss(p - e, x, t, F)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_adam_first_step_and_convergence():
    p = np.array([1.0, -1.0, 0.5])
    g = np.array([0.3, -2.0, 1e-3])
    p1, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), step=1, lr=0.01)
    # bias-corrected first step moves every coordinate by lr against its gradient
    np.testing.assert_allclose(p - p1, 0.01 * np.sign(g), rtol=1e-4)
    # minimise |q - c|^2
    c = np.array([3.0, -2.0, 0.0])
    q, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for s in range(1, 3001):
        q, m, v = mlp.adam(q, 2 * (q - c), m, v, step=s, lr=0.05)
    np.testing.assert_allclose(q, c, atol=1e-3)
