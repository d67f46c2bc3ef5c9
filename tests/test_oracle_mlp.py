"""Pins of the FP64 warm-start references (oracle/mlp.py) against facts that
do not use their own formulas: central finite differences of the loss, the
closed form of Adam's first step, a network with zero hidden weights, and a
snapshot set of known rank for the greedy basis."""
import numpy as np

from oracle import mlp as OM


def _net(rng, dims):
    n = sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))
    return rng.standard_normal(n) * 0.7


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(5)
    dims = [3, 5, 4, 2]
    theta = _net(rng, dims)
    x = rng.standard_normal((6, 3))
    t = rng.standard_normal((6, 2))
    _, g = OM.loss_and_gradient(theta, dims, x, t)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        lp, _ = OM.loss_and_gradient(theta + e, dims, x, t)
        lm, _ = OM.loss_and_gradient(theta - e, dims, x, t)
        fd[i] = (lp - lm) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_zero_hidden_weights_give_the_output_bias():
    dims = [4, 6, 3]
    layers = [(np.zeros((6, 4)), np.zeros(6)), (np.ones((3, 6)), np.array([0.5, -1.0, 2.0]))]
    y, acts = OM.forward(OM.flatten(layers), dims, np.random.default_rng(1).standard_normal((5, 4)))
    assert np.array_equal(y, np.tile([0.5, -1.0, 2.0], (5, 1)))
    assert np.array_equal(acts[1], np.zeros((5, 6)))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = OM.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    assert np.allclose(th1 - th, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_greedy_basis_recovers_a_known_span():
    rng = np.random.default_rng(3)
    D = 40
    Q, _ = np.linalg.qr(rng.standard_normal((D, 3)))
    mean = rng.standard_normal(D)
    C = rng.standard_normal((12, 3)) * np.array([5.0, 2.0, 0.5])
    Y = mean + C @ Q.T
    Phi, picked = OM.greedy_basis(Y, mean, 6)
    assert Phi.shape == (3, D)                      # rank 3: stops after three vectors
    assert np.allclose(Phi @ Phi.T, np.eye(3), atol=1e-12)
    P = Phi.T @ Phi
    assert np.allclose(P @ Q, Q, atol=1e-10)        # spans the same subspace
    Yc = Y - mean
    assert picked[0] == int(np.argmax(np.sum(Yc * Yc, axis=1)))
