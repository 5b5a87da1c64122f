"""Pins for the numpy reference MLP (CPU): the backward pass against central
finite differences of the forward pass, the loss gradient against finite
differences of the loss, and Adam against its closed form on a quadratic."""
import numpy as np

from oracle import mlp_ref

SHAPE = (5, 16, 3, 6)


def test_param_count_matches_layout():
    assert mlp_ref.param_count(5, 64, 3, 6) == 5 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 6 + 6
    p = mlp_ref.init(SHAPE)
    assert p.size == mlp_ref.param_count(*SHAPE)


def test_backward_is_gradient_of_forward():
    rng = np.random.default_rng(0)
    p = mlp_ref.init(SHAPE, seed=1) + rng.normal(0, 0.05, mlp_ref.param_count(*SHAPE))
    x = rng.normal(size=(7, 5))
    dy = rng.normal(size=(7, 6))
    g = mlp_ref.backward(p, SHAPE, x, dy)
    h = 1e-6
    for idx in rng.choice(p.size, 40, replace=False):
        pp = p.copy(); pp[idx] += h
        pm = p.copy(); pm[idx] -= h
        fd = ((mlp_ref.forward(pp, SHAPE, x)[0] - mlp_ref.forward(pm, SHAPE, x)[0]) * dy).sum() / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(fd))


def test_loss_gradient():
    rng = np.random.default_rng(2)
    y = rng.normal(size=(9, 6))
    t = rng.normal(size=(9, 6))
    w = rng.uniform(0.5, 2.0, 6)
    L, dy = mlp_ref.loss(y, t, w)
    h = 1e-6
    for _ in range(10):
        s, o = rng.integers(9), rng.integers(6)
        yp = y.copy(); yp[s, o] += h
        ym = y.copy(); ym[s, o] -= h
        fd = (mlp_ref.loss(yp, t, w)[0] - mlp_ref.loss(ym, t, w)[0]) / (2 * h)
        assert abs(fd - dy[s, o]) < 1e-8


def test_adam_first_step_is_signed_lr():
    # with zero moments, the first bias-corrected step is lr * g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = mlp_ref.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-9)


def test_adam_minimises_quadratic():
    p = np.array([4.0, -3.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 3001):
        p, m, v = mlp_ref.adam(p, 2 * p, m, v, 0.05, 0.9, 0.999, 1e-8, t)
    assert np.abs(p).max() < 1e-2
