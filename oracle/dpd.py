"""ENUF-DPD real-space sum for Slater-type smeared charges (paper Sec. 2.4).

TEST INFRASTRUCTURE ONLY: part of the oracle.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; it imports nothing
from the HIP library or its package.

A Slater density rho_e(r) = q exp(-2r/lambda_e) / (pi lambda_e^3) (Eq. 51)
interacts with another as point charges do, scaled by B_U(r) for the energy
(Eq. 53, 55) and by B_F(r) for the force (Eq. 54, 56), with x = r/lambda_e
(the paper's beta r* with beta = R_c/lambda_e and r* = r/R_c):
    B_U = 1 - (1 + x) exp(-2x),   B_F = 1 - (1 + 2x(1 + x)) exp(-2x).
In ENUF-DPD the factors are applied to the real-space terms only, inside the
real-space cutoff, past which both are close to 1; the reciprocal and self
terms are those of point charges.  So the real-space pair energy is
ke q_i q_j erfc(a r)/r B_U(r), its force the point-charge real-space force
(the negative gradient of erfc(a r)/r) times B_F(r), and the potential
ke q_j erfc(a r)/r B_U(r).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from oracle import ewald as ew


def slater_factors(r, lam):
    """(B_U, B_F) at distances r for decay length lam (Eq. 57-58)."""
    x = np.asarray(r, np.float64) / lam
    e = np.exp(-2.0 * x)
    return 1.0 - (1.0 + x) * e, 1.0 - (1.0 + 2.0 * x * (1.0 + x)) * e


def real_slater(x, q, box, alpha, rc, lam, ke=1.0, sample=None):
    """Real-space energy, forces and potentials of smeared charges over
    minimum-image pairs closer than rc (rc <= min(L)/2).  Plain numpy, one
    row of pairs per particle: every particle for systems of a few thousand,
    or only the rows of ``sample`` (then the energy is returned as nan)."""
    x = np.asarray(x, np.float64)
    q = np.asarray(q, np.float64)
    box = np.asarray(box, np.float64)
    if rc > 0.5 * box.min() * (1 + 1e-12):
        raise ValueError("minimum image needs rc <= min(L)/2")
    n = len(q)
    rows = np.arange(n) if sample is None else np.asarray(sample)
    E = 0.0 if sample is None else float("nan")
    F = np.zeros((len(rows), 3))
    phi = np.zeros(len(rows))
    c2a = 2.0 * alpha / math.sqrt(math.pi)
    for a, i in enumerate(rows):
        d = x[i] - x
        d -= box * np.rint(d / box)
        r = np.sqrt((d * d).sum(1))
        m = (r < rc) & (np.arange(n) != i)
        r, d, qj = r[m], d[m], q[m]
        bu, bf = slater_factors(r, lam)
        u = erfc(alpha * r) / r
        # the point-charge real-space force per unit separation vector,
        # -(d/dr)(erfc(a r)/r) / r
        g = (u + c2a * np.exp(-(alpha * r) ** 2)) / (r * r)
        phi[a] = ke * np.sum(qj * u * bu)
        F[a] = ke * q[i] * np.sum((qj * g * bf)[:, None] * d, axis=0)
        if sample is None:
            E += 0.5 * q[i] * phi[a]
    return E, F, phi


def ewald_slater(x, q, box, alpha, rc, lam, ke=1.0, tol=1e-16):
    """Ewald sum of smeared charges: the real-space part above plus the
    point-charge reciprocal (converged k-set), self and background terms."""
    e_r, f_r, phi_r = real_slater(x, q, box, alpha, rc, lam, ke)
    e_k, f_k, phi_k = ew.recip(x, q, box, alpha, ke, tol=tol)
    e_s, e_b, phi_s, phi_b = ew.self_terms(q, box, alpha, ke)
    return {"E": e_r + e_k + e_s + e_b, "E_R": e_r, "F": f_r + f_k, "F_R": f_r,
            "phi": phi_r + phi_k + phi_s + phi_b, "phi_R": phi_r}
