"""Persistent binning (ENUF_OPT_SKIN): the particle orders of the last sort
are kept across evaluations while no particle has moved more than skin/2.

* Over a random walk of the particles (steps of 0.02, some crossing the
  periodic boundary, cell and tile faces), every evaluation of a persistent
  context equals that of a context that sorts every time, element by
  element (FP64 to rounding, FP32 at the FP32 mirror tolerance), in both
  force modes, with potentials and the adjoint; the sort count shows the
  orders were kept for most steps and rebuilt when the walk went past the
  skin.
* A charge change forces a sort.
* The NVE run of test_gpu_md through persistent binning: the same energy
  conservation, and one sort for the whole run.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2004_12484_amd import enuf, inputs  # noqa: E402

from gpu_util import rms_rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _sorts(eng):
    return int(eng.stage(enuf.STAGE_COUNTS).cpu().numpy()[5])


def _eval(eng, x, q):
    E, F, phi = eng.energy_forces(x, q, potential=True)
    gx, gq = eng.energy_grad(1.0)
    torch.cuda.synchronize()
    return (E.cpu().numpy(), F.double().cpu().numpy(), phi.double().cpu().numpy(), gx.double().cpu().numpy(),
            gq.double().cpu().numpy())


@pytest.mark.parametrize("prec,mode", [("f64", "ik"), ("f64", "analytic"), ("f32", "ik"), ("f32", "analytic")])
def test_persistent_equals_sorting_evaluation(prec, mode):
    rng = np.random.default_rng(61)
    n, box = 3000, np.array([14.0, 15.0, 16.0])
    x = rng.uniform(0, 1, (n, 3)) * box
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * rng.uniform(0.5, 1.5, n)
    q[rng.uniform(size=n) < 0.2] = 0.0
    args = (box, n, 1.0, 3.5, (32, 32, 64), 6)
    # skin 0.45: half of it is under one grid point on every axis (h = 0.25 on z)
    keep = enuf.Enuf(*args, precision=prec, force_mode=mode, skin=0.45)
    ref = enuf.Enuf(*args, precision=prec, force_mode=mode)
    dt = keep.dtype
    qt = to_dev(q, dt)
    tol = 1e-10 if prec == "f64" else 5e-5
    for step in range(30):
        xt = to_dev(x, dt)
        a = _eval(keep, xt, qt)
        b = _eval(ref, xt, qt)
        scale = np.abs(b[0][1:]).sum()
        assert np.abs(a[0] - b[0]).max() <= (1e-11 if prec == "f64" else 3e-5) * scale, (step, a[0], b[0])
        for k in range(1, 5):
            assert rms_rel(a[k], b[k]) <= tol, (step, k, rms_rel(a[k], b[k]))
        # a random walk; positions are not wrapped, so some leave the box
        x = x + rng.normal(scale=0.02, size=x.shape)
    sorts = _sorts(keep)
    print(f"{prec} {mode}: {sorts} sorts in 30 evaluations (sorting context: {_sorts(ref)})")
    assert _sorts(ref) == 30
    assert 2 <= sorts <= 25


def test_charge_change_forces_a_sort():
    rng = np.random.default_rng(62)
    n, box = 1000, np.array([10.0, 10.0, 10.0])
    x = to_dev(rng.uniform(0, 1, (n, 3)) * box, torch.float64)
    qh = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    eng = enuf.Enuf(box, n, 1.0, 3.0, (32, 32, 32), 4, precision="f64", skin=0.5)
    eng.energy_forces(x, to_dev(qh, torch.float64))
    eng.energy_forces(x, to_dev(qh, torch.float64))
    assert _sorts(eng) == 1
    qh[5] = 0.0
    qh[6] = 0.0
    E, F, _ = eng.energy_forces(x, to_dev(qh, torch.float64))
    assert _sorts(eng) == 2
    ref = enuf.Enuf(box, n, 1.0, 3.0, (32, 32, 32), 4, precision="f64")
    E2, F2, _ = ref.energy_forces(x, to_dev(qh, torch.float64))
    assert abs(float(E[0]) - float(E2[0])) <= 1e-11 * abs(float(E2[2]))
    assert rms_rel(F.cpu().numpy(), F2.cpu().numpy()) <= 1e-10
    assert np.all(F.cpu().numpy()[5:7] == 0.0)


def test_skin_option_validation():
    box = np.array([10.0, 10.0, 10.0])
    eng = enuf.Enuf(box, 100, 1.0, 3.0, (32, 32, 32), 8, precision="f64")
    with pytest.raises(enuf.EnufError) as ei:
        eng.set_option(enuf.OPT_SKIN, -1.0)
    assert ei.value.status == enuf.ENUF_EINVAL
    with pytest.raises(enuf.EnufError) as ei:   # p = 8 on 8-point tiles leaves no margin
        eng.set_option(enuf.OPT_SKIN, 0.2)
    assert ei.value.status == enuf.ENUF_EUNSUPPORTED
    e6 = enuf.Enuf(box, 100, 1.0, 3.0, (32, 32, 32), 6, precision="f64")
    e6.set_option(enuf.OPT_SKIN, 0.3)           # one grid point of margin fits
    with pytest.raises(enuf.EnufError) as ei:
        e6.set_option(enuf.OPT_SKIN, 1.0)       # two do not
    assert ei.value.status == enuf.ENUF_EUNSUPPORTED


def test_nve_through_persistent_binning():
    w = inputs.nacl()
    rc = 0.5 * w.box[0]
    alpha = 4.0 / rc

    def run(skin):
        eng = enuf.Enuf(w.box, w.N, alpha, rc, (32, 32, 32), 6, precision="f64", force_mode="analytic", skin=skin)
        x = to_dev(w.x, torch.float64)
        q = to_dev(w.q, torch.float64)
        v = to_dev(np.random.default_rng(5).normal(scale=0.02, size=(w.N, 3)), torch.float64)
        v -= v.mean(0)
        E, F, _ = eng.energy_forces(x, q)
        F = F.clone()
        tot = []
        for _ in range(100):
            v += 0.5 * 0.02 * F
            x = x + 0.02 * v
            E, F, _ = eng.energy_forces(x, q)
            F = F.clone()
            v += 0.5 * 0.02 * F
            tot.append(float(E[0].item()) + 0.5 * float((v * v).sum().item()))
        return np.array(tot), _sorts(eng)

    t0, s0 = run(0.0)
    t1, s1 = run(0.5)
    scale = abs(t0[0])
    print(f"NVE: drift {np.abs(t0 - t0[0]).max():.3e} sorting every step ({s0} sorts), "
          f"{np.abs(t1 - t1[0]).max():.3e} persistent ({s1} sorts)")
    assert s0 == 101 and s1 <= 2
    assert np.abs(t1 - t1[0]).max() <= 1e-5 * scale
    assert np.abs(t1 - t0).max() <= 1e-9 * scale
