"""Pins for the numpy ENUF mirror (the gridding steps of the oracle).

The mirror's pieces are checked against closed forms (the textbook cubic
B-spline, the Poisson-summation link between the window's continuous and
discrete Fourier coefficients), exact identities of the discrete method
(charge conservation of the spread, the quadratic-form identity, zero net
ik force, gradient = finite differences of its own energy, invariance under
whole-grid-step shifts) and against the direct Ewald oracle, which it must
approach as the window widens.
"""
import math

import numpy as np
import pytest

from oracle import enuf_mirror as em
from oracle import ewald as ew
from paper_2004_12484_amd import inputs


def test_cubic_bspline_matches_textbook_basis():
    t = np.linspace(0, 1, 17, endpoint=False)
    w, dw = em.bspline_stencil(t, 4)
    expect = np.stack([(1 - t) ** 3 / 6, (3 * t ** 3 - 6 * t ** 2 + 4) / 6,
                       (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6, t ** 3 / 6], -1)
    assert np.abs(w - expect).max() < 1e-15
    dexp = np.stack([-(1 - t) ** 2 / 2, (9 * t ** 2 - 12 * t) / 6,
                     (-9 * t ** 2 + 6 * t + 3) / 6, t ** 2 / 2], -1)
    assert np.abs(dw - dexp).max() < 1e-14


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_partition_of_unity(p):
    t = np.random.default_rng(p).uniform(0, 1, 1000)
    w, dw = em.bspline_stencil(t, p)
    assert np.abs(w.sum(-1) - 1).max() < 1e-14
    assert np.abs(dw.sum(-1)).max() < 1e-13
    assert (w >= 0).all()


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_window_derivative_is_finite_difference(p):
    t = np.linspace(0.05, 0.95, 9)
    h = 1e-6
    _, dw = em.bspline_stencil(t, p)
    wp, _ = em.bspline_stencil(t + h, p)
    wm, _ = em.bspline_stencil(t - h, p)
    assert np.abs((wp - wm) / (2 * h) - dw).max() < 1e-8


@pytest.mark.parametrize("p", [4, 6])
def test_window_ft_poisson_summation(p):
    # discrete coefficients = sum over aliases of the continuous transform
    M = 32
    cd = em.window_ft(M, p, "discrete")
    n = np.fft.fftfreq(M, 1.0 / M)
    acc = np.zeros(M)
    for r in range(-4000, 4001):
        t = np.pi * (n + r * M) / M
        s = np.where(t == 0, 1.0, np.sin(t) / np.where(t == 0, 1, t))
        acc += s ** p
    assert np.abs(acc - cd).max() < 1e-9
    cc = em.window_ft(M, p, "continuous")
    assert cc[0] == 1.0 and np.all(cc > 0)


def test_spread_conserves_charge_and_hits_nodes():
    box = np.array([5.0, 6.0, 7.0])
    M = (8, 16, 32)
    rng = np.random.default_rng(1)
    x = rng.uniform(-10, 20, (50, 3))
    q = rng.normal(size=50)
    for p in (2, 4, 6):
        rho = em.spread(x, q, box, M, p)
        assert rho.shape == (32, 16, 8)
        assert abs(rho.sum() - q.sum()) < 1e-12
    # p = 2 (linear) puts a charge sitting on a node entirely on that node
    xn = np.array([[3 * box[0] / 8, 5 * box[1] / 16, 31 * box[2] / 32]])
    rho = em.spread(xn, np.array([2.0]), box, M, 2)
    assert rho[31, 5, 3] == pytest.approx(2.0, abs=1e-13)
    assert abs(np.abs(rho).sum() - 2.0) < 1e-12


def test_structure_factor_converges_to_definition():
    # S~(n) = rho^(n)/c(n) -> sum_j q_j exp(-2 pi i n.x_j) as p grows
    box = np.array([4.0, 4.0, 4.0])
    M = (16, 16, 16)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 4, (20, 3))
    q = rng.normal(size=20)
    n = np.array([2, -3, 1])
    u = x / box
    exact = np.sum(q * np.exp(-2j * np.pi * (u @ n)))
    errs = []
    for p in (2, 4, 6, 8):
        rec = em.reciprocal(x, q, box, 1.0, M, p, want_grad=False)
        idx = (n[2] % 16, n[1] % 16, n[0] % 16)
        errs.append(abs(rec["S"][idx] - exact) / abs(exact))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-4


@pytest.mark.parametrize("p", [4, 6])
def test_discrete_energy_identities(p):
    x, q, box = _sys()
    rec = em.reciprocal(x, q, box, 1.1, (16, 16, 32), p)
    # quadratic form: E_K = 1/2 sum q_i phi_i
    assert abs(0.5 * np.dot(q, rec["phi_K"]) - rec["E_K"]) < 1e-12 * abs(rec["E_K"])
    # ik forces conserve momentum exactly
    fk = rec["F_K"]
    assert np.abs(fk.sum(0)).max() < 1e-12 * np.abs(fk).max() * len(q)


def _sys(n=40, seed=4):
    rng = np.random.default_rng(seed)
    box = np.array([6.0, 6.5, 11.0])
    x = rng.uniform(0, 1, (n, 3)) * box
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return x, q, box


def test_gradient_is_exact_derivative_of_discrete_energy():
    x, q, box = _sys()
    M, p, alpha = (16, 16, 32), 6, 1.1
    rec = em.reciprocal(x, q, box, alpha, M, p)
    h = 1e-6
    for i in (0, 7, 33):
        for d in range(3):
            xp = x.copy(); xp[i, d] += h
            xm = x.copy(); xm[i, d] -= h
            ep = em.reciprocal(xp, q, box, alpha, M, p, want_grad=False)["E_K"]
            emi = em.reciprocal(xm, q, box, alpha, M, p, want_grad=False)["E_K"]
            fd = (ep - emi) / (2 * h)
            assert abs(fd - rec["grad_K"][i, d]) < 1e-7 * max(1.0, np.abs(rec["grad_K"]).max())
    for i in (2, 11):
        qp = q.copy(); qp[i] += h
        qm = q.copy(); qm[i] -= h
        fd = (em.reciprocal(x, qp, box, alpha, M, p, want_grad=False)["E_K"]
              - em.reciprocal(x, qm, box, alpha, M, p, want_grad=False)["E_K"]) / (2 * h)
        assert abs(fd - rec["phi_K"][i]) < 1e-7 * max(1.0, abs(fd))


def test_grid_step_shift_invariance():
    x, q, box = _sys()
    M = np.array([16, 16, 32])
    a = em.reciprocal(x, q, box, 1.1, M, 4, want_grad=False)
    b = em.reciprocal(x + 3 * box / M, q, box, 1.1, M, 4, want_grad=False)
    assert abs(a["E_K"] - b["E_K"]) < 1e-12 * abs(a["E_K"])
    assert np.abs(a["F_K"] - b["F_K"]).max() < 1e-11 * np.abs(a["F_K"]).max()


def test_converges_to_direct_ewald_same_modes():
    # against the oracle restricted to the same modes, only the window error
    # remains; it must fall steeply with p
    w = inputs.nacl()
    ref = ew.ewald(w.x, w.q, w.box, w.alpha, w.r_c, kset="modes", M=w.M)
    errs = []
    for p in (2, 4, 6, 8):
        m = em.enuf(w.x, w.q, w.box, w.alpha, w.r_c, w.M, p, want_grad=False)
        errs.append(em.rms_rel(m["F_K"], ref["F_K"]))
        assert abs(m["E"] - ref["E"]) < 1e-3 * abs(ref["E"])
    assert all(b < 0.1 * a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-7


def test_nacl_default_parameters_meet_accuracy_target():
    # default C1 parameters (alpha = 5.6/L, r_c = L/2, M = 32, p = 4):
    # RMS relative force error <= 1e-4 and energy error <= 1e-6 against the
    # converged Ewald sum
    w = inputs.nacl()
    ref = ew.ewald(w.x, w.q, w.box, w.alpha, w.r_c)
    m = em.enuf(w.x, w.q, w.box, w.alpha, w.r_c, w.M, w.p)
    assert em.rms_rel(m["F"], ref["F"]) < 1e-4
    assert abs(m["E"] - ref["E"]) / abs(ref["E"]) < 1e-6
    assert em.rms_rel(-m["grad_x"], ref["F"]) < 1e-4
    assert em.rms_rel(m["phi"], ref["phi"]) < 1e-5


def test_single_charge_background():
    # non-neutral single charge: mirror with a wide window reproduces the
    # Wigner energy (background + self + k-space)
    L = 5.0
    box = np.array([L, L, L])
    x = np.array([[1.0, 2.0, 3.5]])
    q = np.array([1.0])
    m = em.enuf(x, q, box, 6.0 / L, L / 2, (32, 32, 32), 8, want_grad=False)
    expect = -2.837297479480619 / (2 * L)
    assert abs(m["E"] - expect) < 1e-8


# ---- the paper's NFFT form: Gaussian window, oversampling ----------------
def test_gaussian_transform_matches_quadrature():
    """The scaling step's closed form sqrt(pi b) exp(-b (pi n/M)^2) is the
    Fourier transform of exp(-d^2/b): checked by numerical quadrature."""
    from scipy.integrate import quad

    for p, sigma in ((4, 2.0), (6, 1.5), (8, 2.0)):
        b = em.gaussian_shape(p, sigma)
        M = 32
        c = em.window_ft(M, p, ("gaussian", b))
        for n in (0, 3, 7):
            val, _ = quad(lambda d: math.exp(-d * d / b) * math.cos(2 * math.pi * n * d / M), -40, 40,
                          limit=400, epsabs=1e-14)
            assert abs(val - c[n]) < 1e-10 * max(1.0, abs(val))


def test_gaussian_stencil_sum_approaches_its_transform():
    """Poisson summation for the truncated Gaussian stencil: the stencil's
    own Fourier sum at a kept mode equals the continuous transform (times
    the particle's phase) up to the truncation and aliasing error, which
    falls with the cutoff m at fixed oversampling."""
    rng = np.random.default_rng(5)
    M, sigma = 64, 2.0
    K = em.kept_modes(M, sigma)
    n = np.arange(-(K // 2) + 1, K // 2)
    errs = []
    for p in (4, 6, 8):
        b = em.gaussian_shape(p, sigma)
        worst = 0.0
        for s in rng.uniform(0, M, 20):
            fl = math.floor(s)
            w, _ = em.gaussian_stencil(np.array([s - fl]), p, b)
            ls = fl - p // 2 + 1 + np.arange(p)
            disc = (w[0][None, :] * np.exp(-2j * np.pi * n[:, None] * ls[None, :] / M)).sum(1)
            cont = math.sqrt(math.pi * b) * np.exp(-b * (np.pi * n / M) ** 2) * np.exp(-2j * np.pi * n * s / M)
            worst = max(worst, float(np.abs(disc / cont - 1).max()))
        errs.append(worst)
    # (largest at the highest kept mode, where the first alias is nearest)
    assert errs[0] > 5 * errs[1] > 25 * errs[2]
    assert errs[2] < 2e-3


def test_gaussian_window_derivative_is_finite_difference():
    t = np.linspace(0.05, 0.95, 9)
    h = 1e-6
    b = em.gaussian_shape(6, 2.0)
    _, dw = em.gaussian_stencil(t, 6, b)
    wp, _ = em.gaussian_stencil(t + h, 6, b)
    wm, _ = em.gaussian_stencil(t - h, 6, b)
    assert np.abs((wp - wm) / (2 * h) - dw).max() < 1e-8


def test_kept_modes():
    assert em.kept_modes(64, 1.0) == 64 and em.kept_modes(64, 2.0) == 32
    assert em.kept_modes(64, 1.5) == 42 and em.kept_modes(32, 1.5) == 20


def _fig1_system():
    rng = np.random.default_rng(3)
    n = 400
    box = np.array([12.0, 12.0, 12.0])
    x = rng.uniform(0, 1, (n, 3)) * box
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    delta, rc = 1e-5, 6.0
    return x, q, box, math.sqrt(-math.log(delta)) / rc, rc


@pytest.mark.parametrize("sigma", [1.5, 2.0])
def test_gaussian_energy_error_falls_with_m(sigma):
    """The energy error of the oversampled Gaussian form against the Ewald
    sum over the same kept modes falls steeply with the NFFT cutoff m and is
    at the Ewald accuracy (delta = 1e-5) from m = 2 on."""
    x, q, box, alpha, rc = _fig1_system()
    M = 32
    K = em.kept_modes(M, sigma)
    ref = ew.ewald(x, q, box, alpha, rc, kset="modes", M=(K, K, K))
    errs = []
    for m in (1, 2, 3):
        r = em.enuf(x, q, box, alpha, rc, (M, M, M), 2 * m + 2, window="gaussian", sigma=sigma, want_grad=False)
        errs.append(abs(r["E"] - ref["E"]) / abs(ref["E"]))
    assert errs[0] > 10 * errs[1] > 10 * errs[2] / 2
    assert errs[1] < 1e-4 and errs[2] < 1e-5


def test_gaussian_gradient_is_exact_derivative_of_discrete_energy():
    x, q, box = _sys()
    M, p, alpha = (16, 16, 32), 6, 1.1
    rec = em.reciprocal(x, q, box, alpha, M, p, window="gaussian", sigma=2.0)
    h = 1e-6
    for i in (0, 7, 33):
        for d in range(3):
            xp = x.copy(); xp[i, d] += h
            xm = x.copy(); xm[i, d] -= h
            ep = em.reciprocal(xp, q, box, alpha, M, p, window="gaussian", sigma=2.0, want_grad=False)["E_K"]
            emi = em.reciprocal(xm, q, box, alpha, M, p, window="gaussian", sigma=2.0, want_grad=False)["E_K"]
            assert abs((ep - emi) / (2 * h) - rec["grad_K"][i, d]) < 1e-7 * max(1.0, np.abs(rec["grad_K"]).max())
    assert abs(0.5 * np.dot(q, rec["phi_K"]) - rec["E_K"]) < 1e-12 * abs(rec["E_K"])
