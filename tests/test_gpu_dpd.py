"""GPU parity of the ENUF-DPD mode (Slater-type smeared charges, paper
Sec. 2.4, Eq. 51-58): real-space pair terms scaled by B_U (energy,
potential) and B_F (force), reciprocal and self terms of point charges.

Reference = the numpy ENUF mirror's reciprocal, self and background parts
plus the oracle's smeared real-space sum (oracle/dpd.py), both FP64 CPU.
The system is a DPD fluid (density 3 in units of R_c = 1, beta = 1.125, so
lambda_e = 0.889, real-space cutoff 3 R_c), half the beads charged: many
pairs lie closer than lambda_e/2, where the kernel takes the factors'
series form.
* FP64 element by element at the mirror tolerances (summation order only),
  in both reciprocal force modes.
* FP32 within the FP32 bar (RMS 5e-5).
* The adjoint differentiates the scaled energy exactly: dE/dx against
  central differences of the FP64 energy, dE/dq against the potentials.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dpd  # noqa: E402
from oracle import enuf_mirror as em  # noqa: E402

from paper_2004_12484_amd import enuf  # noqa: E402

from gpu_util import rms_rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

LAM = 1.0 / 1.125


def _dpd_system(n=1500, seed=41):
    rng = np.random.default_rng(seed)
    L = (n / 3.0) ** (1.0 / 3.0)
    box = np.array([L, L, L * 1.05])
    x = rng.uniform(0, 1, (n, 3)) * box
    q = np.zeros(n)
    q[: n // 2] = np.where(np.arange(n // 2) % 2 == 0, 1.0, -1.0)
    return x, q, box


def _reference(x, q, box, alpha, rc, M, p):
    m = em.enuf(x, q, box, alpha, rc, M, p, want_grad=False)
    e_r, f_r, phi_r = dpd.real_slater(x, q, box, alpha, rc, LAM)
    return {"E": m["E"] - m["E_R"] + e_r, "E_R": e_r, "F": m["F"] - m["F_R"] + f_r,
            "phi": m["phi"] - m["phi_R"] + phi_r, "F_point": m["F"],
            "scale": abs(e_r) + abs(m["E_K"]) + abs(m["E_self"]) + abs(m["E_bg"])}


def _gpu(x, q, box, alpha, rc, M, p, precision):
    eng = enuf.Enuf(box, len(q), alpha, rc, M, p, precision=precision, slater=LAM)
    E, F, phi = eng.energy_forces(to_dev(x, eng.dtype), to_dev(q, eng.dtype), potential=True)
    torch.cuda.synchronize()
    return eng, E.cpu().numpy(), F.double().cpu().numpy(), phi.double().cpu().numpy()


def test_slater_fp64_vs_mirror():
    x, q, box = _dpd_system()
    alpha, rc, M, p = 0.92, 3.0, (32, 32, 32), 6
    ref = _reference(x, q, box, alpha, rc, M, p)
    _, E, F, phi = _gpu(x, q, box, alpha, rc, M, p, "f64")
    assert abs(E[1] - ref["E_R"]) <= 1e-11 * abs(ref["E_R"])
    assert abs(E[0] - ref["E"]) <= 1e-11 * ref["scale"]
    assert np.linalg.norm(F - ref["F"]) <= 1e-10 * np.linalg.norm(ref["F"])
    assert np.linalg.norm(phi - ref["phi"]) <= 1e-10 * np.linalg.norm(ref["phi"])
    # the smearing moves the forces far beyond those tolerances
    assert np.linalg.norm(ref["F"] - ref["F_point"]) > 1e-2 * np.linalg.norm(ref["F"])


def test_slater_analytic_mode_fp64_vs_mirror():
    # the smeared real-space sum next to the analytic-derivative reciprocal
    # forces (minus the mirror's exact gradient of the discrete energy)
    x, q, box = _dpd_system(seed=45)
    alpha, rc, M, p = 0.92, 3.0, (32, 32, 32), 6
    m = em.enuf(x, q, box, alpha, rc, M, p, want_grad=True)
    e_r, f_r, phi_r = dpd.real_slater(x, q, box, alpha, rc, LAM)
    eng = enuf.Enuf(box, len(q), alpha, rc, M, p, precision="f64", force_mode="analytic", slater=LAM)
    E, F, phi = eng.energy_forces(to_dev(x, eng.dtype), to_dev(q, eng.dtype), potential=True)
    torch.cuda.synchronize()
    ref_f = -m["grad_K"] + f_r
    ref_phi = m["phi"] - m["phi_R"] + phi_r
    assert abs(E.cpu().numpy()[1] - e_r) <= 1e-11 * abs(e_r)
    assert np.linalg.norm(F.cpu().numpy() - ref_f) <= 1e-10 * np.linalg.norm(ref_f)
    assert np.linalg.norm(phi.cpu().numpy() - ref_phi) <= 1e-10 * np.linalg.norm(ref_phi)


def test_slater_fp32_vs_mirror():
    # 4000 beads: three cells per axis, the kernel's fixed-image path (the
    # FP64 case above, two cells per axis, takes the minimum-image one)
    x, q, box = _dpd_system(n=4000, seed=42)
    alpha, rc, M, p = 0.92, 3.0, (32, 32, 32), 6
    xr = x.astype(np.float32).astype(np.float64)
    ref32 = _reference(xr, q, box, alpha, rc, M, p)
    _, E, F, phi = _gpu(x, q, box, alpha, rc, M, p, "f32")
    c = q != 0
    eps_f = rms_rel(F[c], ref32["F"][c])
    eps_p = rms_rel(phi, ref32["phi"])
    print(f"ENUF-DPD fp32: eps_F={eps_f:.3e} eps_phi={eps_p:.3e}")
    assert eps_f <= 5e-5
    assert eps_p <= 5e-5
    assert abs(E[0] - ref32["E"]) <= 1e-5 * ref32["scale"]


def test_slater_adjoint_vs_finite_differences():
    x, q, box = _dpd_system(n=1000, seed=43)
    alpha, rc, M, p = 0.92, 3.0, (16, 16, 16), 6
    eng = enuf.Enuf(box, len(q), alpha, rc, M, p, precision="f64", slater=LAM)
    xt, qt = to_dev(x, torch.float64), to_dev(q, torch.float64)
    _, _, phi = eng.energy_forces(xt, qt, potential=True)
    gx, gq = eng.energy_grad(1.0)
    gx, gq = gx.cpu().numpy(), gq.cpu().numpy()
    assert np.linalg.norm(gq - phi.cpu().numpy()) <= 1e-12 * np.linalg.norm(gq)

    def energy(xx):
        E, _, _ = eng.energy_forces(xx, qt, forces=False)
        return float(E[0].item())

    # charged particles whose charged partners all lie away from the cutoff
    h = 1e-5
    d = x[:, None, :] - x[None, :, :]
    d -= box * np.rint(d / box)
    r = np.sqrt((d * d).sum(-1))
    ch = np.nonzero(q)[0]
    ok = [i for i in ch if np.all(np.abs(r[i, ch] - rc) > 4 * h)][:12]
    assert len(ok) == 12
    fd = np.zeros((len(ok), 3))
    for a, i in enumerate(ok):
        for k in range(3):
            xp = xt.clone()
            xp[i, k] += h
            xm = xt.clone()
            xm[i, k] -= h
            fd[a, k] = (energy(xp) - energy(xm)) / (2 * h)
    err = rms_rel(gx[ok], fd)
    print(f"ENUF-DPD adjoint vs FD: {err:.3e}")
    assert err <= 1e-6


def test_slater_option_validation_and_reset():
    x, q, box = _dpd_system(n=1000, seed=44)
    alpha, rc, M, p = 0.92, 3.0, (16, 16, 16), 6
    eng = enuf.Enuf(box, len(q), alpha, rc, M, p, precision="f64")
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(enuf.EnufError) as ei:
            eng.set_option(enuf.OPT_SLATER, bad)
        assert ei.value.status == enuf.ENUF_EINVAL
    xt, qt = to_dev(x, torch.float64), to_dev(q, torch.float64)
    _, F0, _ = eng.energy_forces(xt, qt)
    F0 = F0.cpu().numpy()
    eng.set_option(enuf.OPT_SLATER, LAM)
    _, F1, _ = eng.energy_forces(xt, qt)
    F1 = F1.cpu().numpy()
    # back to point charges: the first result again (up to summation order)
    eng.set_option(enuf.OPT_SLATER, 0.0)
    _, F2, _ = eng.energy_forces(xt, qt)
    F2 = F2.cpu().numpy()
    assert np.linalg.norm(F1 - F0) > 1e-2 * np.linalg.norm(F0)
    assert np.linalg.norm(F2 - F0) <= 1e-13 * np.linalg.norm(F0)
