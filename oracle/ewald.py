"""FP64 direct Ewald oracle (Python side of ``ewald_direct.c``).

TEST INFRASTRUCTURE ONLY: the oracle of the ENUF hot path.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it.  It
imports nothing from the HIP library or its package.

The Ewald sum is the plain definition that ENUF approximates (paper
Sec. 2.1): U = U^R + U^K + U^self (Eq. 25), with U^R the erfc pair sum
inside the cutoff (Eq. 17), U^K the k-space sum over the structure factor
(Eq. 22 and 26), U^self from Eq. 24, plus a neutralising-background term for
non-neutral systems (zero when sum q = 0; the paper assumes neutrality).
Forces are -dU/dr (Eq. 27-28), potentials dU/dq.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ewald_direct.c")
_LIB = os.path.join(_HERE, "libewald_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, i64, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_real_images.argtypes = [i64, vp, vp, vp, d, d, d, vp, vp, vp]
        lib.oracle_real_minimage.argtypes = [i64, vp, vp, vp, d, d, d, i64, vp, vp, vp, vp]
        lib.oracle_real_minimage.restype = ctypes.c_int
        lib.oracle_real_cells_energy.argtypes = [i64, vp, vp, vp, d, d, d, vp]
        lib.oracle_real_cells_energy.restype = ctypes.c_int
        lib.oracle_recip.restype = ctypes.c_int
        lib.oracle_recip.argtypes = [i64, vp, vp, vp, d, d, vp, d, i64, vp, vp, vp, vp]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(x, q, box):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    if x.shape[0] != q.shape[0]:
        raise ValueError("x and q disagree on N")
    return x, q, box


def real_images(x, q, box, alpha, rc, ke=1.0):
    """Real-space sum with explicit periodic images (Eq. 16 cut at rc)."""
    x, q, box = _prep(x, q, box)
    n = x.shape[0]
    e = np.zeros(1)
    f = np.zeros((n, 3))
    phi = np.zeros(n)
    _load().oracle_real_images(n, _p(x), _p(q), _p(box), alpha, rc, ke, _p(e), _p(f), _p(phi))
    return float(e[0]), f, phi


def real_minimage(x, q, box, alpha, rc, ke=1.0, sample=None, energy=True):
    """Real-space sum, minimum image (requires rc <= min(L)/2).  With
    energy=False the O(N^2) pair energy is skipped (returned as nan) and only
    the sampled forces and potentials are computed."""
    x, q, box = _prep(x, q, box)
    if rc > 0.5 * box.min() * (1 + 1e-12):
        raise ValueError("minimum image needs rc <= min(L)/2")
    n = x.shape[0]
    if sample is None:
        ns, sp = -1, None
        m = n
    else:
        sp = np.ascontiguousarray(sample, dtype=np.int64)
        ns, m = sp.shape[0], sp.shape[0]
    e = np.zeros(1)
    f = np.zeros((m, 3))
    phi = np.zeros(m)
    rc_ = _load().oracle_real_minimage(n, _p(x), _p(q), _p(box), alpha, rc, ke, ns, _p(sp),
                                       _p(e) if energy else None, _p(f), _p(phi))
    if rc_ != 0:
        raise MemoryError("oracle_real_minimage: allocation failed")
    return (float(e[0]) if energy else float("nan")), f, phi


def real_energy_cells(x, q, box, alpha, rc, ke=1.0):
    """Real-space pair energy (Eq. 17, minimum image) over all charged
    pairs, the pairs enumerated with a linked-cell list (at least 3 cells
    per axis; otherwise the all-pairs loop of real_minimage).  Same sum as
    real_minimage's energy, in another order: for systems too large for the
    all-pairs loop."""
    x, q, box = _prep(x, q, box)
    if rc > 0.5 * box.min() * (1 + 1e-12):
        raise ValueError("minimum image needs rc <= min(L)/2")
    e = np.zeros(1)
    rc_ = _load().oracle_real_cells_energy(x.shape[0], _p(x), _p(q), _p(box), alpha, rc, ke, _p(e))
    if rc_ == -2:
        return real_minimage(x, q, box, alpha, rc, ke, sample=np.zeros(0, np.int64))[0]
    if rc_ != 0:
        raise MemoryError("oracle_real_cells_energy: allocation failed")
    return float(e[0])


def kset_converged(box, alpha, tol=1e-16):
    """Sphere k^2 <= kcut^2 with exp(-kcut^2/4a^2) = tol, and the per-axis
    mode bound it implies."""
    kcut2 = 4.0 * alpha * alpha * math.log(1.0 / tol)
    nmax = [int(math.floor(math.sqrt(kcut2) * L / (2 * math.pi))) for L in box]
    return np.array(nmax, np.int32), kcut2


def recip(x, q, box, alpha, ke=1.0, nmax=None, kcut2=None, tol=1e-16, sample=None):
    """k-space sum over explicit vectors (Eq. 22, 26; force of Eq. 41)."""
    x, q, box = _prep(x, q, box)
    if nmax is None:
        nmax, kc = kset_converged(box, alpha, tol)
        if kcut2 is None:
            kcut2 = kc
    nmax = np.ascontiguousarray(nmax, dtype=np.int32)
    if kcut2 is None:
        kcut2 = 0.0
    n = x.shape[0]
    if sample is None:
        ns, sp, m = -1, None, n
    else:
        sp = np.ascontiguousarray(sample, dtype=np.int64)
        ns, m = sp.shape[0], sp.shape[0]
    e = np.zeros(1)
    f = np.zeros((m, 3))
    phi = np.zeros(m)
    rc = _load().oracle_recip(n, _p(x), _p(q), _p(box), alpha, ke, _p(nmax), float(kcut2),
                              ns, _p(sp), _p(e), _p(f), _p(phi))
    if rc != 0:
        raise MemoryError("oracle_recip: allocation failed")
    return float(e[0]), f, phi


def self_terms(q, box, alpha, ke=1.0):
    """Self energy (Eq. 24, entering Eq. 25 with a minus sign) and the
    neutralising-background energy, with their charge derivatives."""
    q = np.asarray(q, np.float64)
    V = float(np.prod(box))
    Q = float(q.sum())
    Q2 = float((q * q).sum())
    e_self = -ke * alpha / math.sqrt(math.pi) * Q2
    e_bg = -ke * math.pi * Q * Q / (2.0 * V * alpha * alpha)
    phi_self = -2.0 * ke * alpha / math.sqrt(math.pi) * q
    phi_bg = np.full(q.shape, -ke * math.pi * Q / (V * alpha * alpha))
    return e_self, e_bg, phi_self, phi_bg


def ewald(x, q, box, alpha, rc, ke=1.0, kset="converged", tol=1e-16, M=None,
          sample=None, real="minimage"):
    """Full Ewald sum.  Returns a dict with E (total) and its parts
    E_R, E_K, E_self, E_bg; F and phi for the sampled particles (all when
    ``sample`` is None), with their real/reciprocal parts.

    kset="converged": every k with exp(-k^2/4a^2) >= tol (the reference).
    kset="modes": the cube |n_d| <= M_d/2 - 1 (the modes a grid M keeps).
    """
    x, q, box = _prep(x, q, box)
    if real == "images":
        if sample is not None:
            raise ValueError("images mode computes every particle")
        e_r, f_r, phi_r = real_images(x, q, box, alpha, rc, ke)
    else:
        e_r, f_r, phi_r = real_minimage(x, q, box, alpha, rc, ke, sample)
    if kset == "converged":
        e_k, f_k, phi_k = recip(x, q, box, alpha, ke, tol=tol, sample=sample)
    elif kset == "modes":
        nmax = np.array([m // 2 - 1 for m in M], np.int32)
        e_k, f_k, phi_k = recip(x, q, box, alpha, ke, nmax=nmax, kcut2=0.0, sample=sample)
    else:
        raise ValueError(kset)
    e_s, e_b, phi_s, phi_b = self_terms(q, box, alpha, ke)
    idx = np.arange(len(q)) if sample is None else np.asarray(sample)
    return {
        "E": e_r + e_k + e_s + e_b, "E_R": e_r, "E_K": e_k, "E_self": e_s, "E_bg": e_b,
        "F": f_r + f_k, "F_R": f_r, "F_K": f_k,
        "phi": phi_r + phi_k + phi_s[idx] + phi_b[idx], "phi_R": phi_r, "phi_K": phi_k,
        "sample": idx,
    }


def energy(x, q, box, alpha, rc, ke=1.0, tol=1e-16):
    """Total energy only (no per-particle outputs)."""
    return ewald(x, q, box, alpha, rc, ke, tol=tol, sample=np.zeros(0, np.int64))["E"]
