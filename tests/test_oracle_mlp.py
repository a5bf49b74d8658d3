"""Pins of the FP64 cost-model network: hand-written backprop vs central differences."""
import numpy as np

from oracle import mlp


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(5, seed=1)
    X = rng.standard_normal((17, 5))
    t = rng.standard_normal(17)
    _, g = mlp.loss_and_grad(p, X, t)
    eps = 1e-6
    for k in p:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp, _ = mlp.loss_and_grad(p, X, t)
            flat[idx] = old - eps
            lm, _ = mlp.loss_and_grad(p, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].ravel()[idx]
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9


def test_adam_fits_a_smooth_function():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(256, 3))
    t = np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    p = mlp.init_params(3, seed=0)
    st = {}
    l0, _ = mlp.loss_and_grad(p, X, t)
    for _ in range(800):
        _, g = mlp.loss_and_grad(p, X, t)
        p = mlp.adam_step(p, g, st, lr=3e-3)
    l1, _ = mlp.loss_and_grad(p, X, t)
    assert l1 < 0.05 * l0
