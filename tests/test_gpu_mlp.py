"""GPU: the parameter-predictor kernels against the numpy FP64 reference
(forward, loss, backward, Adam), and a training run that fits a smooth map."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp_ref  # noqa: E402
from paper_2004_12484_amd import mlp  # noqa: E402

pytestmark = pytest.mark.gpu

SHAPE = (5, 64, 3, 6)
# FP32 dot products of length <= 64 through 4 layers: relative rounding ~1e-6;
# 1e-5 of the output / gradient scale bounds it with margin.
TOL = 1e-5


def _data(B=100, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(B, 5)).astype(np.float32), rng.normal(size=(B, 6)).astype(np.float32)


@pytest.mark.parametrize("B", [1, 31, 32, 100, 1000])
def test_forward_matches_reference(B):
    net = mlp.MLP(*SHAPE, seed=3)
    x, _ = _data(B)
    y = net.forward(torch.tensor(x)).cpu().numpy()
    yr, _ = mlp_ref.forward(net.numpy_params().astype(np.float64), SHAPE, x.astype(np.float64))
    assert np.abs(y - yr).max() <= TOL * max(1.0, np.abs(yr).max())


@pytest.mark.parametrize("B", [1, 33, 257])
def test_loss_and_backward_match_reference(B):
    net = mlp.MLP(*SHAPE, seed=4)
    x, t = _data(B, seed=B)
    w = np.linspace(0.5, 2.0, 6).astype(np.float32)
    loss = net.loss_and_grad(torch.tensor(x), torch.tensor(t), torch.tensor(w))
    p64 = net.numpy_params().astype(np.float64)
    y, _ = mlp_ref.forward(p64, SHAPE, x.astype(np.float64))
    L, dy = mlp_ref.loss(y, t, w)
    g = mlp_ref.backward(p64, SHAPE, x.astype(np.float64), dy)
    assert abs(float(loss.item()) - L) <= TOL * max(1.0, L)
    gg = net.grad.cpu().numpy()
    assert np.abs(gg - g).max() <= TOL * max(1e-3, np.abs(g).max())


def test_adam_matches_reference():
    net = mlp.MLP(*SHAPE, seed=5)
    rng = np.random.default_rng(6)
    p = net.numpy_params().astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, 4):
        g = rng.normal(size=p.size).astype(np.float32)
        net.grad.copy_(torch.tensor(g))
        net.adam_step(lr=1e-3)
        p, m, v = mlp_ref.adam(p, g.astype(np.float64), m, v, 1e-3, 0.9, 0.999, 1e-8, t)
    assert np.abs(net.numpy_params() - p).max() <= 1e-6


def test_training_reduces_loss_on_smooth_map():
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (4096, 5)).astype(np.float32)
    T = np.stack([np.sin(X[:, 0]) + X[:, 1] * X[:, 2], X[:, 3] ** 2, np.tanh(X[:, 4] - X[:, 0]),
                  X.sum(1) / 5, X[:, 1] - X[:, 3], np.cos(X[:, 2])], 1).astype(np.float32)
    net = mlp.MLP(*SHAPE, seed=8)
    hist = net.fit(X, T, np.ones(6, np.float32), epochs=40, batch=256, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0]
    y = net.forward(torch.tensor(X)).cpu().numpy()
    assert float(((y - T) ** 2).mean()) < 2e-3
