"""Pins for the oracle MLP (CPU only)."""

import numpy as np

from oracle import mlp
from paper_1505_07959_amd import inputs


def _batch(S=5, seed=0):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((S, 6))
    Bm = rng.standard_normal((S, 8, 8))
    G = np.einsum("sab,scb->sac", Bm, Bm) + 0.1 * np.eye(8)
    b = rng.standard_normal((S, 8))
    f = rng.uniform(1.0, 2.0, size=S)
    c_base = np.tile(np.array([1.0, -1.0, 0, 0, 0.3, -0.2, 0.1, 0.05]), (S, 1))
    return Z, c_base, G, b, f


def test_param_count():
    assert mlp.n_params() == 9288
    assert inputs.mlp_init(1).shape == (9288,)


def test_backward_matches_finite_differences():
    Z, c_base, G, b, f = _batch()
    rng = np.random.default_rng(3)
    theta = inputs.mlp_init(2) + 0.05 * rng.standard_normal(mlp.n_params())
    L, g = mlp.loss_grad(theta, Z, c_base, G, b, f, rho=0.3)
    idx = rng.choice(theta.size, size=40, replace=False)
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = 1e-6
        fd = (mlp.loss(theta + e, Z, c_base, G, b, f, rho=0.3)
              - mlp.loss(theta - e, Z, c_base, G, b, f, rho=0.3)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_output_layer_is_euler():
    Z, c_base, G, b, f = _batch()
    Y, _ = mlp.forward(inputs.mlp_init(4), Z)
    assert np.all(Y == 0.0)


def test_adam_decreases_loss():
    Z, c_base, G, b, f = _batch(S=32, seed=5)
    theta = inputs.mlp_init(6)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = mlp.loss(theta, Z, c_base, G, b, f)
    for t in range(1, 201):
        L, g = mlp.loss_grad(theta, Z, c_base, G, b, f)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 1e-3)
    assert mlp.loss(theta, Z, c_base, G, b, f) < 0.5 * L0


def test_adam_first_step_is_signed_lr():
    """With bias correction, the first Adam step moves every parameter with a
    non-zero gradient by lr * sign(g) (up to eps)."""
    theta = np.zeros(5)
    g = np.array([3.0, -2.0, 1e-3, -7.0, 0.0])
    th, m, v = mlp.adam_step(theta, g, np.zeros(5), np.zeros(5), 1, 0.01, eps=1e-12)
    assert np.allclose(th, -0.01 * np.sign(g), atol=1e-9)
