"""Pins of the ENUF-DPD oracle (Slater-type smeared charges, paper Sec. 2.4)
against what the physics and the paper fix, independently of its formulas:

* B_U from Gauss's law: the potential of the Slater density of Eq. 51,
  integrated numerically (enclosed charge over r plus the outer shells),
  equals q B_U(r)/r (Eq. 52-53).
* B_F from B_U: for the unscreened interaction the force is minus the
  derivative of the energy, so B_F/r^2 = -d/dr (B_U/r) (Eq. 54 from Eq. 53),
  checked by central differences.
* The limits of Eq. 59-60: U -> q_i q_j beta/R_c = q_i q_j/lambda_e and
  F -> 0 as r -> 0; both factors tend to 1 far from the charge.
* The real-space sum reduces to the point-charge oracle (itself pinned in
  test_oracle.py) as lambda_e -> 0, and its forces sum to zero.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import dpd
from oracle import ewald as ew


@pytest.mark.parametrize("lam", [0.5, 0.8889, 2.0])
def test_slater_potential_from_gauss_law(lam):
    rho = lambda s: math.exp(-2.0 * s / lam) / (math.pi * lam ** 3)  # unit charge
    for r in (0.05, 0.3, 1.0, 2.5, 6.0):
        inner = integrate.quad(lambda s: 4 * math.pi * s * s * rho(s), 0.0, r, epsabs=0, epsrel=1e-13)[0]
        outer = integrate.quad(lambda s: 4 * math.pi * s * rho(s), r, np.inf, epsabs=0, epsrel=1e-13)[0]
        phi = inner / r + outer
        bu, _ = dpd.slater_factors(r, lam)
        assert abs(bu / r - phi) <= 1e-10 * phi


@pytest.mark.parametrize("lam", [0.5, 0.8889, 2.0])
def test_slater_force_is_minus_energy_derivative(lam):
    h = 1e-5
    for r in (0.1, 0.5, 1.0, 2.0, 4.0):
        up = dpd.slater_factors(r + h, lam)[0] / (r + h)
        um = dpd.slater_factors(r - h, lam)[0] / (r - h)
        f = dpd.slater_factors(r, lam)[1] / (r * r)
        assert abs(-(up - um) / (2 * h) - f) <= 1e-8 * max(abs(f), 1e-3)


def test_slater_limits_eq59_eq60():
    beta, Rc = 1.125, 1.0
    lam = Rc / beta
    r = 1e-4
    bu, bf = dpd.slater_factors(r, lam)
    assert abs(bu / r - beta / Rc) <= 1e-3 * beta / Rc      # Eq. 59, U(0) = q_i q_j beta / R_c
    assert abs(bf / (r * r)) <= 1e-3                        # Eq. 60, F(0) = 0
    assert dpd.slater_factors(1e-6, lam)[1] / 1e-12 < bf / (r * r)
    # both factors approach 1 away from the charge (near 1 at 3 R_c, the
    # paper's real-space cutoff; to 1e-12 by 16 lambda_e)
    bu3, bf3 = dpd.slater_factors(3 * Rc, lam)
    assert 0.99 < bu3 < 1 and 0.96 < bf3 < 1
    bu16, bf16 = dpd.slater_factors(16 * lam, lam)
    assert abs(1 - bu16) < 1e-12 and abs(1 - bf16) < 1e-11


def _system(n=120, L=9.0, seed=7):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, L, (n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return x, q, np.array([L, L, L * 1.1])


def test_real_slater_point_charge_limit():
    x, q, box = _system()
    e, f, phi = dpd.real_slater(x, q, box, 0.7, 4.0, 1e-6)
    e0, f0, phi0 = ew.real_minimage(x, q, box, 0.7, 4.0)
    assert abs(e - e0) <= 1e-12 * abs(e0)
    assert np.abs(f - f0).max() <= 1e-12 * np.abs(f0).max()
    assert np.abs(phi - phi0).max() <= 1e-12 * np.abs(phi0).max()


def test_real_slater_newton_and_samples():
    x, q, box = _system()
    e, f, phi = dpd.real_slater(x, q, box, 0.7, 4.0, 0.8889)
    assert np.abs(f.sum(0)).max() <= 1e-11 * np.abs(f).max()
    assert abs(e - 0.5 * np.dot(q, phi)) <= 1e-12 * abs(e)
    s = np.array([3, 50, 7])
    _, fs, ps = dpd.real_slater(x, q, box, 0.7, 4.0, 0.8889, sample=s)
    assert np.array_equal(fs, f[s]) and np.array_equal(ps, phi[s])
