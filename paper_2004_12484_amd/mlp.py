"""Binding and training loop of the ENUF parameter predictor
(`include/enuf_mlp.h`).  Every forward, loss, backward and Adam step runs in
the library's HIP kernels; this module only marshals tensors and loops.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import enuf

MLP_EXPORTS = ("enuf_mlp_param_count", "enuf_mlp_cache_count", "enuf_mlp_forward", "enuf_mlp_loss",
               "enuf_mlp_workspace_bytes", "enuf_mlp_backward", "enuf_mlp_adam")


class _Shape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("n_out", ctypes.c_int32)]


_bound = False


def _lib():
    global _bound
    lib = enuf.load_library()
    if not _bound:
        vp, i64, f32, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_int32, ctypes.c_size_t
        sp = ctypes.POINTER(_Shape)
        lib.enuf_mlp_param_count.argtypes = [sp]
        lib.enuf_mlp_param_count.restype = i64
        lib.enuf_mlp_cache_count.argtypes = [sp]
        lib.enuf_mlp_cache_count.restype = i64
        lib.enuf_mlp_forward.argtypes = [sp, vp, i64, vp, vp, vp, vp]
        lib.enuf_mlp_forward.restype = i32
        lib.enuf_mlp_loss.argtypes = [sp, i64, vp, vp, vp, vp, vp, vp]
        lib.enuf_mlp_loss.restype = i32
        lib.enuf_mlp_workspace_bytes.argtypes = [sp, i64]
        lib.enuf_mlp_workspace_bytes.restype = sz
        lib.enuf_mlp_backward.argtypes = [sp, vp, i64, vp, vp, vp, vp, vp, sz, vp]
        lib.enuf_mlp_backward.restype = i32
        lib.enuf_mlp_adam.argtypes = [i64, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
        lib.enuf_mlp_adam.restype = i32
        _bound = True
    return lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _ok(st):
    if st != 0:
        raise enuf.EnufError(st, "MLP kernel call failed")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class MLP:
    """n_in -> n_layers x n_hidden tanh -> n_out, FP32 parameters on the GPU."""

    def __init__(self, n_in=5, n_hidden=64, n_layers=3, n_out=6, params=None, seed=0, device="cuda"):
        self.shape = _Shape(n_in, n_hidden, n_layers, n_out)
        self.dims = (n_in, n_hidden, n_layers, n_out)
        self.device = torch.device(device)
        n = int(_lib().enuf_mlp_param_count(ctypes.byref(self.shape)))
        if n < 0:
            raise ValueError("bad MLP shape")
        if params is None:
            rng = np.random.default_rng(seed)
            parts = []
            d = [n_in] + [n_hidden] * n_layers + [n_out]
            for i, o in zip(d[:-1], d[1:]):
                lim = np.sqrt(6.0 / (i + o))
                parts += [rng.uniform(-lim, lim, o * i), np.zeros(o)]
            params = np.concatenate(parts)
        params = np.asarray(params, np.float32).ravel()
        if params.size != n:
            raise ValueError(f"expected {n} parameters, got {params.size}")
        self.params = torch.tensor(params, device=self.device)
        self.n_params = n
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.t = 0

    def forward(self, x, cache=False):
        x = x.to(self.device, torch.float32).contiguous()
        B = x.shape[0]
        y = torch.empty((B, self.dims[3]), dtype=torch.float32, device=self.device)
        c = None
        if cache:
            nc = int(_lib().enuf_mlp_cache_count(ctypes.byref(self.shape)))
            c = torch.empty((B, nc), dtype=torch.float32, device=self.device)
        _ok(_lib().enuf_mlp_forward(ctypes.byref(self.shape), _p(self.params), B, _p(x), _p(y), _p(c), _stream()))
        return (y, c) if cache else y

    def loss_and_grad(self, x, t, w):
        """Weighted MSE of the batch; leaves d(loss)/d(params) in self.grad."""
        lib = _lib()
        x = x.to(self.device, torch.float32).contiguous()
        t = t.to(self.device, torch.float32).contiguous()
        w = w.to(self.device, torch.float32).contiguous()
        B = x.shape[0]
        y, c = self.forward(x, cache=True)
        dy = torch.empty_like(y)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        _ok(lib.enuf_mlp_loss(ctypes.byref(self.shape), B, _p(y), _p(t), _p(w), _p(dy), _p(loss), _stream()))
        nbytes = int(lib.enuf_mlp_workspace_bytes(ctypes.byref(self.shape), B))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _ok(lib.enuf_mlp_backward(ctypes.byref(self.shape), _p(self.params), B, _p(x), _p(c), _p(dy),
                                  _p(self.grad), _p(ws), nbytes, _stream()))
        return loss

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        _ok(_lib().enuf_mlp_adam(self.n_params, _p(self.params), _p(self.grad), _p(self.m), _p(self.v),
                                 lr, beta1, beta2, eps, self.t, _stream()))

    def fit(self, X, T, W, epochs=200, batch=512, lr=2e-3, lr_final=1e-4, seed=0, log=None):
        """Mini-batch Adam on (X, T) with output weights W; cosine-decayed lr.
        Returns the per-epoch mean training loss."""
        X = torch.as_tensor(X, dtype=torch.float32, device=self.device)
        T = torch.as_tensor(T, dtype=torch.float32, device=self.device)
        W = torch.as_tensor(W, dtype=torch.float32, device=self.device)
        n = X.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        total = epochs * ((n + batch - 1) // batch)
        step = 0
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(self.device)
            acc = torch.zeros((), dtype=torch.float64, device=self.device)
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                loss = self.loss_and_grad(X[idx], T[idx], W)
                frac = step / max(1, total - 1)
                lr_t = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * frac))
                self.adam_step(lr_t)
                acc += loss[0] * idx.numel()
                step += 1
            hist.append(float(acc.item()) / n)
            if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
                log(f"epoch {ep}: loss {hist[-1]:.4e}")
        return hist

    def numpy_params(self):
        return self.params.detach().cpu().numpy().astype(np.float32)
