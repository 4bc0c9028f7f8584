"""Pins for the MLP oracle: central finite differences of the loss, the
loss at a known point, Adam's first step (|update| = lr), the rank rule."""
import numpy as np

from oracle import mlp


def _setup(seed=0, F=6, H=5, R=4, n=7):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.nparams(F, H, R)) * 0.5
    X = rng.standard_normal((n, F))
    T = rng.standard_normal((n, R))
    return theta, X, T, F, H, R


def test_gradient_matches_finite_differences():
    theta, X, T, F, H, R = _setup()
    loss, g = mlp.loss_and_grad(theta, X, T, F, H, R)
    h = 1e-6
    num = np.zeros_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        num[k] = (mlp.loss_and_grad(theta + e, X, T, F, H, R)[0] - mlp.loss_and_grad(theta - e, X, T, F, H, R)[0]) / (2 * h)
    assert np.abs(num - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_loss_at_zero_weights_is_mean_square_target():
    theta, X, T, F, H, R = _setup(1)
    assert abs(mlp.loss_and_grad(np.zeros_like(theta), X, T, F, H, R)[0] - np.mean(T * T)) < 1e-14


def test_adam_first_step_has_magnitude_lr():
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 3.0, -0.1])
    t1, m, v = mlp.adam_step(theta, g, np.zeros(5), np.zeros(5), 1, lr=0.01)
    assert np.allclose(np.abs(t1), 0.01, rtol=1e-6)
    assert np.all(np.sign(t1) == -np.sign(g))


def test_rank_rule():
    z = np.array([[0.0, -3.0, -5.0, -7.0], [1.0, 1.0, 1.0, 1.0], [-9.0, -9.0, -9.0, -9.0]])
    assert mlp.rank_rule(z, thr=-4.0, lmax=8).tolist() == [3, 8, 1]
    assert mlp.rank_rule(z, thr=-4.0, lmax=2).tolist() == [2, 2, 1]
