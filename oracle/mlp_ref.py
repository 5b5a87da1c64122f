"""Reference multilayer perceptron in numpy FP64 (parameter predictor).

TEST INFRASTRUCTURE ONLY: the CPU reference the HIP forward, loss, backward
and Adam kernels are checked against.  Only the tests may import it.

Network: n_in -> n_layers x (n_hidden, tanh) -> n_out (linear).  Parameters
in one flat array, layer by layer: W_l as [out][in] row-major, then b_l.
Backward is written out by the chain rule; it is pinned by finite
differences in the tests.
"""
from __future__ import annotations

import numpy as np


def layer_sizes(n_in, n_hidden, n_layers, n_out):
    dims = [n_in] + [n_hidden] * n_layers + [n_out]
    return list(zip(dims[:-1], dims[1:]))


def param_count(n_in, n_hidden, n_layers, n_out):
    return sum(o * i + o for i, o in layer_sizes(n_in, n_hidden, n_layers, n_out))


def unpack(params, shape):
    out = []
    off = 0
    for i, o in layer_sizes(*shape):
        W = params[off: off + o * i].reshape(o, i)
        off += o * i
        b = params[off: off + o]
        off += o
        out.append((W, b))
    return out


def forward(params, shape, x):
    """Returns (y, activations) with activations[l] the input of layer l."""
    params = np.asarray(params, np.float64)
    a = np.asarray(x, np.float64)
    acts = [a]
    layers = unpack(params, shape)
    for l, (W, b) in enumerate(layers):
        z = a @ W.T + b
        a = np.tanh(z) if l < len(layers) - 1 else z
        acts.append(a)
    return a, acts


def loss(y, t, w):
    """Weighted MSE: sum_{s,o} w_o (y - t)^2 / B and its gradient in y."""
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    w = np.asarray(w, np.float64)
    B = y.shape[0]
    d = y - t
    return float((w[None, :] * d * d).sum() / B), 2.0 * w[None, :] * d / B


def backward(params, shape, x, dy):
    """Gradient of sum(dy * y) with respect to the flat parameter array."""
    params = np.asarray(params, np.float64)
    y, acts = forward(params, shape, x)
    layers = unpack(params, shape)
    grads = []
    dz = np.asarray(dy, np.float64)
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        a_in = acts[l]
        gW = dz.T @ a_in
        gb = dz.sum(0)
        grads.append((gW, gb))
        if l > 0:
            da = dz @ W
            dz = da * (1.0 - a_in * a_in)  # tanh' = 1 - tanh^2
    flat = []
    for gW, gb in reversed(grads):
        flat.append(gW.ravel())
        flat.append(gb)
    return np.concatenate(flat)


def adam(p, g, m, v, lr, b1, b2, eps, t):
    """One Adam step (Kingma & Ba 2015) with bias correction; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init(shape, seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in layer_sizes(*shape):
        lim = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-lim, lim, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)
