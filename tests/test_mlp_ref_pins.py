"""Pins of the FP64 MLP reference: analytic gradient vs central differences,
and a hand-computed one-hidden-unit case of SiLU's derivative."""
import numpy as np

from oracle import mlp_ref


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = rng.normal(0, 0.08, 148481)
    X = rng.normal(0, 1, (12, 64))
    y = rng.normal(0, 1, 12)
    loss, g = mlp_ref.loss_and_grad(P, X, y)
    idx = np.concatenate([rng.choice(16384, 6), 16384 + rng.choice(256, 3), 16640 + rng.choice(65536, 6),
                          82432 + rng.choice(65536, 6), 147968 + rng.choice(256, 3),
                          148224 + rng.choice(256, 4), [148480]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (mlp_ref.loss_and_grad(Pp, X, y)[0] - mlp_ref.loss_and_grad(Pm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_silu_derivative_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp_ref.silu(z + h) - mlp_ref.silu(z - h)) / (2 * h)
    assert np.allclose(mlp_ref.silu_grad(z), fd, atol=1e-9)
    assert mlp_ref.silu(0.0) == 0.0 and abs(mlp_ref.silu_grad(0.0) - 0.5) < 1e-15
