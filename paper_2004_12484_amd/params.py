"""ENUF parameter selection: (alpha, M per axis, p, r_c) for a target RMS
force error.

Three selectors:
  heuristic   the paper's relations (Eq. 31-32), in the library
              (enuf_select_params): fix the target delta and the
              reciprocal cutoff n_c, take alpha from Eq. 31 and r_c from
              Eq. 32, and raise n_c until r_c fits a short-range cutoff
              (Sec. 2.3.2); the grid holds modes up to n_c
  grid search the fastest setting whose measured error meets the target, from
              a sweep of the method itself (sweep.py)
  mlp         a 5 -> 3x64 -> 6 network (mlp.py kernels) trained on those
              sweeps; enuf_select_params evaluates it from data/param_mlp.bin

Features: (log10 N, Ly/Lx, Lz/Lx, charged fraction, log10 target error).
Targets:  (alpha a, log2 Mx, log2 My, log2 Mz, p, r_c / a), a = (V/N)^(1/3).
"""
from __future__ import annotations

import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "data", "param_mlp.npz")
MODEL_BIN = os.path.join(HERE, "data", "param_mlp.bin")   # the same network for enuf_select_params
P_CHOICES = (4, 6, 8)
M_MIN, M_MAX = 8, 512
# the systems the network was trained on (inputs.random_system): outside
# these ranges its prediction is not used
# (densities were drawn from [0.1, 3]; the bound admits 5% beyond, which
# takes in the one-million-bead systems at 2^20 / 70^3 = 3.06)
TRAIN_RANGE = {"N": (1000, 4194304), "density": (0.1, 3.15), "f_q": (0.02, 1.0), "target": (3e-5, 1e-3)}
TRAIN_SHAPES = ((1.0, 1.0), (1.0, 2.0))   # (Ly/Lx, Lz/Lx) of the training boxes


def spacing(N, box):
    return (float(np.prod(box)) / N) ** (1.0 / 3.0)


def features(N, box, f_q, target):
    box = np.asarray(box, float)
    return np.array([math.log10(N), box[1] / box[0], box[2] / box[0], f_q, math.log10(target)], np.float64)


def snap(box, N, alpha_a, log2M, p, rc_a):
    """Valid setting from continuous predictions: M a power of two in
    [8, 512] (rounded up), p in {4, 6, 8} with 2p <= M, r_c <= min(L)/2."""
    box = np.asarray(box, float)
    a = spacing(N, box)
    alpha = float(alpha_a) / a
    M = [int(min(M_MAX, max(M_MIN, 2 ** math.ceil(float(v) - 1e-6)))) for v in log2M]
    pp = min(P_CHOICES, key=lambda c: abs(c - float(p)))
    while any(2 * pp > m for m in M):
        pp -= 2
    rc = min(float(rc_a) * a, 0.5 * float(box.min()))
    return {"alpha": alpha, "M": tuple(M), "p": int(pp), "r_c": rc}


def select_params(N, box, f_q, target, model_path=None):
    """enuf_select_params (C ABI): the Eq. 31-32 heuristic when model_path is
    None, else the network file's prediction (evaluated on the current GPU by
    the MLP kernels) for systems inside its training ranges, the heuristic
    outside them.  Returns (setting, method) with method "heuristic" or
    "network"."""
    import ctypes

    from . import enuf

    lib = enuf.load_library()
    b = (ctypes.c_double * 3)(*[float(v) for v in box])
    alpha, rc = ctypes.c_double(), ctypes.c_double()
    M = (ctypes.c_int32 * 3)()
    p, method = ctypes.c_int32(), ctypes.c_int32()
    path = None if model_path is None else os.fsencode(model_path)
    st = lib.enuf_select_params(b, int(N), float(f_q), float(target), path, ctypes.byref(alpha), ctypes.byref(rc),
                                M, ctypes.byref(p), ctypes.byref(method))
    if st != 0:
        raise enuf.EnufError(st, lib.enuf_select_last_error().decode(errors="replace"))
    s = {"alpha": alpha.value, "M": tuple(int(m) for m in M), "p": int(p.value), "r_c": rc.value}
    return s, ("network" if method.value == 1 else "heuristic")


def heuristic(N, box, f_q, target):
    """Eq. 31-32 (computed by the library): exp(-pi^2 n_c^2/(alpha L)^2) =
    delta and erfc(alpha r_c) ~ exp(-alpha^2 r_c^2) = delta; n_c is raised
    from 2 until r_c <= 3 mean spacings.  The grid keeps modes |n| <= n_c."""
    return select_params(N, box, f_q, target)[0]


def export_bin(npz_path=MODEL_PATH, out=None):
    """Write the network in the flat little-endian file enuf_select_params
    reads (magic, dims, normalisation, training ranges and box shapes,
    parameters)."""
    import struct

    d = np.load(npz_path)
    out = out or os.path.splitext(npz_path)[0] + ".bin"
    dims = [int(v) for v in d["dims"]]
    r = TRAIN_RANGE
    rng = [r["N"][0], r["N"][1], r["density"][0], r["density"][1], r["f_q"][0], r["f_q"][1],
           r["target"][0], r["target"][1]]
    params = np.ascontiguousarray(d["params"], dtype="<f4")
    with open(out, "wb") as f:
        f.write(b"ENUFMLP1")
        f.write(struct.pack("<4i", *dims))
        for k in ("x_mean", "x_std", "y_mean", "y_std"):
            f.write(np.ascontiguousarray(d[k], dtype="<f8").tobytes())
        f.write(struct.pack("<8d", *rng))
        f.write(struct.pack("<i", len(TRAIN_SHAPES)))
        for sh in TRAIN_SHAPES:
            f.write(struct.pack("<2d", *sh))
        f.write(struct.pack("<q", params.size))
        f.write(params.tobytes())
    return out


class Predictor:
    """Trained network plus its feature/target normalisation."""

    def __init__(self, path=MODEL_PATH, device="cuda"):
        from . import mlp

        d = np.load(path)
        self.bin_path = os.path.splitext(path)[0] + ".bin"
        self.xm, self.xs, self.ym, self.ys = d["x_mean"], d["x_std"], d["y_mean"], d["y_std"]
        dims = tuple(int(v) for v in d["dims"])
        self.net = mlp.MLP(*dims, params=d["params"], device=device)

    def predict_raw(self, F):
        import torch

        Xn = (np.atleast_2d(F) - self.xm) / self.xs
        Y = self.net.forward(torch.tensor(Xn, dtype=torch.float32)).cpu().numpy().astype(np.float64)
        return Y * self.ys + self.ym

    def select(self, N, box, f_q, target):
        """The network's setting through enuf_select_params (the heuristic's
        when the system lies outside the training ranges)."""
        return select_params(N, box, f_q, target, model_path=self.bin_path)[0]


def in_training_range(N, box, f_q, target):
    box = np.asarray(box, float)
    rho = N / float(np.prod(box))
    shape = (box[1] / box[0], box[2] / box[0])
    ok_shape = any(abs(shape[0] - a) < 1e-6 and abs(shape[1] - b) < 1e-6 for a, b in TRAIN_SHAPES)
    r = TRAIN_RANGE
    return (ok_shape and r["N"][0] <= N <= r["N"][1] and r["density"][0] <= rho <= r["density"][1]
            and r["f_q"][0] <= f_q <= r["f_q"][1] and r["target"][0] <= target <= r["target"][1])


def choose(x, q, box, target, predictor=None):
    """Setting for one system: the network's prediction when the system lies
    inside its training range, else (the fallback) a grid search over a sweep
    of this very system.  Returns (setting, info)."""
    import time

    q = np.asarray(q)
    N = len(q)
    f_q = float(np.count_nonzero(q)) / N
    if predictor is not None and in_training_range(N, box, f_q, target):
        t0 = time.perf_counter()
        s = predictor.select(N, box, f_q, target)
        return s, {"method": "network", "select_ms": (time.perf_counter() - t0) * 1e3}
    from .sweep import combine, sweep_arrays

    t0 = time.perf_counter()
    rec = sweep_arrays(x, q, box)
    best = grid_search({"settings": combine(rec)}, target)
    info = {"method": "grid_search", "select_ms": (time.perf_counter() - t0) * 1e3,
            "search_gpu_ms": rec["cost_ms"], "settings_tried": int(len(rec["rows"]))}
    if best is None:
        raise RuntimeError("no swept setting meets the target")
    info["expected_err"] = best["err"]
    return {k: best[k] for k in ("alpha", "r_c", "M", "p")}, info


def grid_search(sweep_row, target):
    """Fastest measured setting meeting `target` in one system's sweep record
    (see sweep.py); None when no setting meets it."""
    best = None
    for s in sweep_row["settings"]:
        if s["err"] <= target and (best is None or s["time"] < best["time"]):
            best = s
    return best
