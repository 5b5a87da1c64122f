"""Seeded synthetic workloads for the ENUF hot path.

This module only draws positions, charges and box shapes and records the
run parameters (alpha, r_c, grid, window order) each workload is evaluated
with.  It holds none of the method's arithmetic: no window, no transform, no
Ewald term.  Both the CPU oracle (through the tests) and the HIP path (through
the tests and the benchmark) take their inputs from here, so the two sides see
bit-identical data.

The paper's own systems (ionic-liquid and DPD electrolytes, polyelectrolytes,
dendrimers; Sec. 2.4 and Sec. 4) are not public files.  The generators below
stand in for them with the shapes, sizes and charge patterns of the workloads
the ENUF hot path is measured on:

  nacl        rock-salt crystal, 4x4x4 conventional cells (512 ions), a=5.64,
              optional Gaussian displacement noise (the Madelung set-up of the
              alpha trials, Sec. 2.4.2)
  electrolyte bulk 1:1 point-charge electrolyte, uniform random positions
  charged_fluid  mesoscopic bead fluid, a fraction of the beads charged +-1
  ions_1m     the same geometry with every bead charged: one million ions
  anisotropic orthorhombic box with +1 bead chains (random walks), -1
              counterions and neutral solvent
  random_system  random neutral systems for the parameter-selection sweeps

All generators use numpy's PCG64 (``default_rng(seed)``), draw in float64 and
return C-contiguous arrays.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload",
    "nacl",
    "electrolyte",
    "charged_fluid",
    "ions_1m",
    "anisotropic",
    "random_system",
    "workload",
    "WORKLOADS",
]


@dataclasses.dataclass
class Workload:
    """A seeded system plus the ENUF parameters it is evaluated with."""

    name: str
    x: np.ndarray          # [N,3] float64 positions (not necessarily wrapped)
    q: np.ndarray          # [N] float64 charges
    box: np.ndarray        # [3] float64 box lengths (Lx, Ly, Lz)
    alpha: float           # Ewald splitting parameter
    r_c: float             # real-space cutoff
    M: tuple               # FFT grid (Mx, My, Mz)
    p: int                 # window stencil width per axis
    precision: str         # "f64" or "f32"
    seed: int
    ke: float = 1.0        # Coulomb prefactor 1/(4 pi eps0 eps_r)

    @property
    def N(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_charged(self) -> int:
        return int(np.count_nonzero(self.q))


def _wrap(x: np.ndarray, box: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.mod(x, box[None, :]))


def nacl(cells: int = 4, a: float = 5.64, noise: float = 0.02, seed: int = 1,
         alpha_L: float = 5.6, M: int = 32, p: int = 4,
         precision: str = "f64") -> Workload:
    """Rock-salt crystal of ``cells**3`` conventional cells (8 ions each).

    Na+ on the fcc sites (0,0,0), (0,1/2,1/2), (1/2,0,1/2), (1/2,1/2,0); Cl- on
    the same sites shifted by (1/2,0,0).  Each coordinate gets N(0, (noise*a)^2)
    displacement; ``noise=0`` gives the perfect lattice.  alpha = alpha_L / L,
    r_c = L/2.
    """
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)
    cl = fcc + np.array([.5, 0, 0])
    idx = np.stack(np.meshgrid(np.arange(cells), np.arange(cells),
                               np.arange(cells), indexing="ij"), -1).reshape(-1, 3)
    na_pos = (idx[:, None, :] + fcc[None]).reshape(-1, 3)
    cl_pos = (idx[:, None, :] + cl[None]).reshape(-1, 3)
    x = np.concatenate([na_pos, cl_pos]) * a
    q = np.concatenate([np.ones(len(na_pos)), -np.ones(len(cl_pos))])
    L = cells * a
    box = np.array([L, L, L])
    if noise > 0:
        rng = np.random.default_rng(seed)
        x = x + rng.normal(0.0, noise * a, size=x.shape)
    x = _wrap(x, box)
    return Workload("nacl", x, np.ascontiguousarray(q), box, alpha_L / L, L / 2,
                    (M, M, M), p, precision, seed)


def electrolyte(N: int = 32768, density: float = 0.5, seed: int = 2,
                r_c: float = 3.0, alpha_rc: float = 3.2, M: int = 64, p: int = 4,
                precision: str = "f64") -> Workload:
    """Bulk 1:1 electrolyte: first half +1, second half -1, uniform positions."""
    if N % 2:
        raise ValueError("N must be even for a neutral 1:1 electrolyte")
    L = (N / density) ** (1.0 / 3.0)
    box = np.array([L, L, L])
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(N, 3)) * box[None, :]
    q = np.concatenate([np.ones(N // 2), -np.ones(N // 2)])
    return Workload("electrolyte", _wrap(x, box), q, box, alpha_rc / r_c, r_c,
                    (M, M, M), p, precision, seed)


def charged_fluid(N: int = 1 << 20, L: float = 70.0, charged_fraction: float = 0.2,
                  seed: int = 3, r_c: float = 3.0, alpha: float = 1.0,
                  M: int = 128, p: int = 6, precision: str = "f32") -> Workload:
    """Mesoscopic bead fluid: uniform beads, a seeded subset charged +-1.

    The number of charged beads is ``round(f*N)`` rounded down to even; half
    of them +1, half -1, chosen by a seeded permutation.
    """
    box = np.array([L, L, L], float)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(N, 3)) * box[None, :]
    nq = int(round(charged_fraction * N)) // 2 * 2
    q = np.zeros(N)
    sel = rng.permutation(N)[:nq]
    q[sel[: nq // 2]] = 1.0
    q[sel[nq // 2:]] = -1.0
    return Workload("charged_fluid", _wrap(x, box), q, box, alpha, r_c,
                    (M, M, M), p, precision, seed)


def ions_1m(N: int = 1 << 20, L: float = 70.0, seed: int = 3, r_c: float = 1.8, alpha: float = 2.9 / 1.8,
            M: int = 256, p: int = 6, precision: str = "f32") -> Workload:
    """One million ions: the charged-fluid geometry (uniform positions, same
    seed) with every bead charged, half +1 and half -1 by a seeded
    permutation.  The default (alpha, r_c, M, p) is the fastest FP32 setting
    of a timed grid search (both force modes) whose RMS force error against
    the oracle is <= 1e-4 with margin; it is meant for the analytic-derivative
    force mode."""
    box = np.array([L, L, L], float)
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(N, 3)) * box[None, :]
    q = np.empty(N)
    sel = rng.permutation(N)
    q[sel[: N // 2]] = 1.0
    q[sel[N // 2:]] = -1.0
    return Workload("ions_1m", _wrap(x, box), q, box, alpha, r_c, (M, M, M), p, precision, seed)


def anisotropic(N: int = 1 << 22, box=(120.0, 120.0, 240.0), chain_fraction: float = 0.02,
                chain_len: int = 32, bond: float = 1.0, seed: int = 5,
                r_c: float = 3.0, alpha: float = 1.0, M=(256, 256, 512), p: int = 6,
                precision: str = "f32") -> Workload:
    """Orthorhombic box: +1 bead chains, -1 counterions, neutral solvent.

    ``chain_fraction*N`` sites (rounded down to whole chains) are +1 beads
    on seeded random walks with unit steps in uniformly random directions;
    the same number of -1 counterions are placed uniformly; every other site
    is a neutral solvent bead placed uniformly.
    """
    box = np.asarray(box, float)
    rng = np.random.default_rng(seed)
    n_chains = int(chain_fraction * N) // chain_len
    n_plus = n_chains * chain_len
    starts = rng.uniform(0.0, 1.0, size=(n_chains, 3)) * box[None, :]
    v = rng.normal(size=(n_chains, chain_len - 1, 3))
    v *= bond / np.linalg.norm(v, axis=-1, keepdims=True)
    chains = np.concatenate([starts[:, None, :], starts[:, None, :] + np.cumsum(v, axis=1)], axis=1)
    rest = rng.uniform(0.0, 1.0, size=(N - n_plus, 3)) * box[None, :]
    x = np.concatenate([chains.reshape(-1, 3), rest])
    q = np.zeros(N)
    q[:n_plus] = 1.0
    q[n_plus:2 * n_plus] = -1.0
    return Workload("anisotropic", _wrap(x, box), q, box, alpha, r_c,
                    tuple(M), p, precision, seed)


def random_system(seed: int, n_min: int = 1000, n_max: int = 262144, fq_min: float = 0.05,
                  rho_min: float = 0.1, rho_max: float = 3.0) -> Workload:
    """Random neutral system for the parameter-selection sweeps.

    N log-uniform in [n_min, n_max]; cubic or 1:1:2 box (equal odds); number
    density log-uniform in [rho_min, rho_max]; charged fraction uniform in
    [fq_min, 1]; charges +-1 in equal numbers.  The ENUF parameters recorded
    here are a placeholder (the sweep sets its own).
    """
    rng = np.random.default_rng(seed)
    N = int(round(10 ** rng.uniform(math.log10(n_min), math.log10(n_max))))
    aspect = np.array([1.0, 1.0, 2.0]) if rng.uniform() < 0.5 else np.ones(3)
    density = 10 ** rng.uniform(math.log10(rho_min), math.log10(rho_max))
    fq = rng.uniform(fq_min, 1.0)
    V = N / density
    Lx = (V / np.prod(aspect)) ** (1.0 / 3.0)
    box = Lx * aspect
    x = rng.uniform(0.0, 1.0, size=(N, 3)) * box[None, :]
    nq = max(2, int(round(fq * N)) // 2 * 2)
    q = np.zeros(N)
    sel = rng.permutation(N)[:nq]
    q[sel[: nq // 2]] = 1.0
    q[sel[nq // 2:]] = -1.0
    a = density ** (-1.0 / 3.0)
    return Workload("random_system", _wrap(x, box), q, box, 3.0 / (3.0 * a), 3.0 * a,
                    (32, 32, 32 if aspect[2] == 1 else 64), 4, "f32", seed)


WORKLOADS = {
    "nacl": nacl,
    "electrolyte": electrolyte,
    "charged_fluid": charged_fluid,
    "ions_1m": ions_1m,
    "anisotropic": anisotropic,
}


def workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
