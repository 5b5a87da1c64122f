"""Full-size GPU checks at the benchmark workloads, against stored oracle
values (tests/golden/, written by make_oracle_golden.py from the oracle
alone) on seeded samples of particles, plus the finite-difference check of
the adjoint on the 1M-bead fluid.

* charged_fluid (1M beads, 20% charged, M = 128^3, p = 6, FP32, ik forces):
  sampled forces against the Ewald sum at the same (alpha, r_c) and against
  the converged Coulomb force, and the total energy.
* ions_1m (1M ions, M = 256^3, p = 6, FP32, analytic forces, the bench
  setting): sampled forces against the converged Coulomb force.
* anisotropic (4M sites in 120 x 120 x 240: +1 chains, -1 counterions,
  neutral solvent; FP32, ik forces and potentials at every site) at the
  setting the parameter selector picks for the FP32 bar 5e-4: sampled forces
  and potentials against the converged Coulomb values.  At this size the
  counting sort uses more buckets than at one million particles (an average
  bucket within the fine pass's register path); both sorted orders are
  checked to be permutations of all sites.
* dpd_slater (the 1M-bead fluid as ENUF-DPD: Slater-smeared charges,
  lambda_e = 1/1.125): sampled forces and potentials against the stored
  oracle values (point-charge k-space part plus the smeared real-space sum).
* Autograd at the 1M-bead geometry: the adjoint's dE/dx and dE/dq against
  central finite differences (h = 1e-4) of the FP64-mode energy on 64 seeded
  particles with no pair within 2h of the cutoff, and the FP32 adjoint
  against the FP64 adjoint.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2004_12484_amd import enuf, inputs  # noqa: E402

from gpu_util import rms_rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    return np.load(os.path.join(GOLDEN, f"{name}_oracle.npz"))


def _forces(w, mode="ik", potential=False, precision=None):
    prec = precision or w.precision
    eng = enuf.Enuf(w.box, w.N, w.alpha, w.r_c, w.M, w.p, precision=prec, force_mode=mode)
    E, F, phi = eng.energy_forces(to_dev(w.x, eng.dtype), to_dev(w.q, eng.dtype), potential=potential)
    torch.cuda.synchronize()
    return eng, E.cpu().numpy(), F.double().cpu().numpy(), (phi.double().cpu().numpy() if phi is not None else None)


def test_charged_fluid_fp32_vs_oracle_samples():
    w = inputs.charged_fluid(alpha=0.95)
    g = _golden("charged_fluid")
    assert int(g["N"]) == w.N and np.isclose(float(g["alpha"]), w.alpha)
    _, E, F, _ = _forces(w)
    s = g["sample"]
    eps = rms_rel(F[s], g["F"])
    eps_conv = rms_rel(F[s], g["F_conv"])
    eps_e = abs(E[0] - float(g["E"])) / abs(float(g["E"]))
    print(f"charged_fluid fp32: eps_F={eps:.3e} (converged {eps_conv:.3e}) eps_E={eps_e:.3e}")
    assert eps <= 1e-4
    assert eps_conv <= 1e-4
    assert eps_e <= 1e-3


def test_ions_1m_bench_setting_vs_oracle_samples():
    w = inputs.ions_1m()
    g = _golden("ions_1m")
    _, _, F, _ = _forces(w, mode="analytic")
    eps = rms_rel(F[g["sample"]], g["F_conv"])
    print(f"ions_1m fp32 analytic: eps_F={eps:.3e}")
    assert eps <= 1e-4


def test_anisotropic_4m_vs_oracle_samples():
    w = inputs.anisotropic()
    g = _golden("anisotropic")
    assert int(g["N"]) == w.N and int(g["seed"]) == w.seed
    eng = enuf.Enuf(w.box, w.N, 0.7466666666666666, 4.6875, (128, 128, 256), 4, precision="f32",
                    force_mode="ik")
    E, F, phi = eng.energy_forces(to_dev(w.x, eng.dtype), to_dev(w.q, eng.dtype), potential=True)
    torch.cuda.synchronize()
    s = g["sample"]
    eps_f = rms_rel(F.double().cpu().numpy()[s], g["F_conv"])
    eps_p = rms_rel(phi.double().cpu().numpy()[s], g["phi_conv"])
    print(f"anisotropic 4M fp32: eps_F={eps_f:.3e} eps_phi={eps_p:.3e}")
    assert eps_f <= 5e-4
    assert eps_p <= 5e-4
    counts = eng.stage(enuf.STAGE_COUNTS).cpu().numpy()
    assert counts[0] == w.N
    for st in (enuf.STAGE_SORTED, enuf.STAGE_CELLS):
        perm = np.sort(eng.stage(st).cpu().numpy()[: w.N])
        assert np.array_equal(perm, np.arange(w.N))


def test_dpd_slater_1m_vs_oracle_samples():
    w = inputs.charged_fluid(alpha=0.95)
    g = _golden("dpd_slater")
    assert int(g["N"]) == w.N and np.isclose(float(g["alpha"]), w.alpha) and np.isclose(float(g["r_c"]), w.r_c)
    eng = enuf.Enuf(w.box, w.N, w.alpha, w.r_c, w.M, w.p, precision="f32", force_mode="ik",
                    slater=float(g["slater"]))
    E, F, phi = eng.energy_forces(to_dev(w.x, eng.dtype), to_dev(w.q, eng.dtype), potential=True)
    torch.cuda.synchronize()
    s = g["sample"]
    Fs = F.double().cpu().numpy()[s]
    ps = phi.double().cpu().numpy()[s]
    eps_f = rms_rel(Fs, g["F"])
    eps_p = rms_rel(ps, g["phi"])
    print(f"dpd_slater fp32: eps_F={eps_f:.3e} eps_phi={eps_p:.3e}")
    # the smearing shrinks the real-space forces (the sampled force norm
    # drops ~3x) but leaves the reciprocal part, and the method's error in
    # it, unchanged: the bar of the point-charge run holds in absolute terms
    gp = _golden("charged_fluid")
    assert np.array_equal(gp["sample"], s)
    assert np.linalg.norm(Fs - g["F"]) <= 1e-4 * np.linalg.norm(gp["F"])
    assert np.linalg.norm(ps - g["phi"]) <= 1e-4 * np.linalg.norm(gp["phi"])
    assert eps_f <= 3e-4


def _fd_sample(w, k, h, rng):
    """k charged particles whose every charged partner lies farther than 2h
    from the cutoff sphere (the real-space energy jumps there)."""
    charged = np.nonzero(w.q)[0]
    xc = w.x[charged]
    out = []
    for i in rng.permutation(charged):
        d = xc - w.x[i]
        d -= w.box * np.rint(d / w.box)
        r = np.sqrt((d * d).sum(1))
        r = r[r > 0]
        if np.all(np.abs(r - w.r_c) > 2 * h) and r.min() > 0.5:
            out.append(i)
            if len(out) == k:
                break
    return np.array(out)


def test_autograd_1m_fluid_vs_finite_differences():
    h = 1e-4
    w = inputs.charged_fluid(alpha=0.95, precision="f64")
    eng = enuf.Enuf(w.box, w.N, w.alpha, w.r_c, w.M, w.p, precision="f64")
    x = to_dev(w.x, torch.float64)
    q = to_dev(w.q, torch.float64)
    eng.energy_forces(x, q, potential=True)
    gx, gq = eng.energy_grad(1.0)
    gx, gq = gx.cpu().numpy(), gq.cpu().numpy()
    sample = _fd_sample(w, 64, h, np.random.default_rng(64))
    assert len(sample) == 64

    def energy(xt, qt):
        E, _, _ = eng.energy_forces(xt, qt, forces=False)
        return float(E[0].item())

    fdx = np.zeros((len(sample), 3))
    fdq = np.zeros(len(sample))
    for a, i in enumerate(sample):
        for d in range(3):
            xp = x.clone()
            xp[i, d] += h
            xm = x.clone()
            xm[i, d] -= h
            fdx[a, d] = (energy(xp, q) - energy(xm, q)) / (2 * h)
        qp = q.clone()
        qp[i] += h
        qm = q.clone()
        qm[i] -= h
        fdq[a] = (energy(x, qp) - energy(x, qm)) / (2 * h)
    ex = rms_rel(gx[sample], fdx)
    eq = rms_rel(gq[sample], fdq)
    print(f"1M fluid adjoint vs FD: dE/dx {ex:.3e}, dE/dq {eq:.3e}")
    # E is quadratic in q, so the q difference is exact but for rounding: E's
    # parts are ~1e5 here, rounded at ~1e-16 relative (~1e-11), divided by
    # 2h = 2e-4 against potentials of O(10): ~1e-8 relative; positions add
    # the O(h^2) truncation of the window polynomials
    assert ex <= 1e-6
    assert eq <= 1e-7
    # the FP32 adjoint against the FP64 one on the same FP32-rounded inputs
    # (rounding the positions alone moves the forces of the closest pairs by
    # ~2 ulp(x)/r, ~1e-3 for r ~ 0.01)
    x32 = to_dev(w.x, torch.float32)
    q32 = to_dev(w.q, torch.float32)
    eng.energy_forces(x32.double(), q32.double(), potential=True)
    gx64, gq64 = eng.energy_grad(1.0)
    e32 = enuf.Enuf(w.box, w.N, w.alpha, w.r_c, w.M, w.p, precision="f32")
    e32.energy_forces(x32, q32, potential=True)
    gx32, gq32 = e32.energy_grad(1.0)
    c = w.q != 0
    ex32 = rms_rel(gx32.double().cpu().numpy()[c], gx64.cpu().numpy()[c])
    eq32 = rms_rel(gq32.double().cpu().numpy(), gq64.cpu().numpy())
    print(f"1M fluid FP32 adjoint vs FP64 adjoint: dE/dx {ex32:.3e}, dE/dq {eq32:.3e}")
    assert ex32 <= 5e-5
    assert eq32 <= 5e-5
