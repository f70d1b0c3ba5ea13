"""The FP64 reference network: gradient against central finite differences."""
import numpy as np

from oracle import mlp


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(mlp.n_params()) * 0.2
    X = rng.standard_normal((7, 16))
    T = rng.standard_normal((7, 6))
    loss, g = mlp.loss_and_grad(theta, X, T)
    idx = rng.choice(len(theta), 40, replace=False)
    # include every block: first/last weights and biases
    idx = np.concatenate([idx, [0, 16 * 128, 16 * 128 + 127, len(theta) - 1, len(theta) - 7]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss_and_grad(theta + e, X, T)[0] - mlp.loss_and_grad(theta - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_layout_size():
    assert mlp.n_params() == 16 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 6 + 6
