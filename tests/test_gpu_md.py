"""Energy and momentum conservation in short NVE runs (velocity Verlet,
unit masses) driven by the library's forces: the paper's claim that ENUF
keeps total energy and momentum, checked on the two force modes.

* analytic mode: the forces are the exact negative gradient of the computed
  energy, so the total energy's excursion is the integrator's own, which
  shrinks as dt^2 (halving dt over the same time divides it by ~4).
* ik mode (the paper's Eq. 41-42): the forces sum to zero up to rounding,
  so the total momentum stays at its initial value.

System: the perturbed rock-salt crystal (512 ions) with alpha r_c = 4 so
that pairs crossing the real-space cutoff change the energy by ~1e-9 only;
FP64.  The integration itself is test code (torch arithmetic on the device);
every force evaluation goes through the library.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2004_12484_amd import enuf, inputs  # noqa: E402

from gpu_util import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _nve(mode, dt, t_end, seed=5):
    w = inputs.nacl()
    rc = 0.5 * w.box[0]
    alpha = 4.0 / rc
    eng = enuf.Enuf(w.box, w.N, alpha, rc, (32, 32, 32), 6, precision="f64", force_mode=mode)
    x = to_dev(w.x, torch.float64)
    q = to_dev(w.q, torch.float64)
    v = to_dev(np.random.default_rng(seed).normal(scale=0.02, size=(w.N, 3)), torch.float64)
    v -= v.mean(0)
    E, F, _ = eng.energy_forces(x, q)
    F = F.clone()
    tot, mom = [], []
    for _ in range(int(round(t_end / dt))):
        v += 0.5 * dt * F
        x = x + dt * v
        E, F, _ = eng.energy_forces(x, q)
        F = F.clone()
        v += 0.5 * dt * F
        tot.append(float(E[0].item()) + 0.5 * float((v * v).sum().item()))
        mom.append(v.sum(0).cpu().numpy())
    E0 = tot[0]
    return np.array(tot) - E0, np.array(mom), abs(E0)


def test_analytic_forces_conserve_energy_to_integrator_order():
    d1, _, scale = _nve("analytic", 0.02, 2.0)
    d2, _, _ = _nve("analytic", 0.01, 2.0)
    a1, a2 = np.abs(d1).max(), np.abs(d2).max()
    print(f"NVE analytic: max |dE| {a1:.3e} (dt 0.02), {a2:.3e} (dt 0.01), |E| {scale:.3e}")
    assert a1 <= 1e-5 * scale
    assert 3.0 <= a1 / a2 <= 5.0


def test_ik_forces_conserve_momentum():
    _, mom, _ = _nve("ik", 0.02, 2.0)
    drift = np.abs(mom - mom[0]).max()
    print(f"NVE ik: momentum drift {drift:.3e}")
    assert drift <= 1e-10
