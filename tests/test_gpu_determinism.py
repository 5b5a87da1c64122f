"""Deterministic mode (ENUF_OPT_DETERMINISTIC): the same inputs give bitwise
the same energies, forces and potentials from run to run.

Two contexts evaluate the same system, on different streams and with other
work between their calls (so the sort's LDS atomics interleave differently);
with the option every result is bitwise equal, in FP64 and FP32, in both
force modes, for a uniform system and for a clustered one whose bins exceed
the one-thread ordering (the workgroup path).  The deterministic results
equal the default mode's to rounding.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2004_12484_amd import enuf  # noqa: E402

from gpu_util import rms_rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _system(clustered, seed=81):
    rng = np.random.default_rng(seed)
    n, box = 6000, np.array([12.0, 13.0, 14.0])
    x = rng.uniform(0, 1, (n, 3)) * box
    if clustered:
        # a third of the particles in a 1.5^3 corner: bins of hundreds
        k = n // 3
        x[:k] = rng.uniform(0, 1.5, (k, 3)) + 3.0
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * rng.uniform(0.5, 1.5, n)
    return x, q, box


def _eval(eng, x, q, stream):
    with torch.cuda.stream(stream):
        E, F, phi = eng.energy_forces(x, q, potential=True)
        gx, gq = eng.energy_grad(1.0)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (E, F, phi, gx, gq)]


@pytest.mark.parametrize("clustered", [False, True])
@pytest.mark.parametrize("prec,mode", [("f64", "ik"), ("f64", "analytic"), ("f32", "ik"), ("f32", "analytic")])
def test_bitwise_reproducible(prec, mode, clustered):
    x, q, box = _system(clustered)
    dt = torch.float64 if prec == "f64" else torch.float32
    args = (box, len(q), 1.1, 3.5, (32, 32, 64), 6)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    engs = []
    for s in (s1, s2):
        with torch.cuda.stream(s):
            e = enuf.Enuf(*args, precision=prec, force_mode=mode)
            e.set_option(enuf.OPT_DETERMINISTIC, 1)
        engs.append(e)
    xt, qt = to_dev(x, dt), to_dev(q, dt)
    a = _eval(engs[0], xt, qt, s1)
    # other work in between, on the other stream
    noise = torch.randn(1 << 20, device="cuda")
    for _ in range(3):
        noise = noise * 1.0001
    b = _eval(engs[1], xt, qt, s2)
    c = _eval(engs[0], xt, qt, s1)
    for u, v, w in zip(a, b, c):
        assert np.array_equal(u, v) and np.array_equal(u, w)
    assert engs[0].flags() == 0
    # the default mode differs only in summation order
    ref = enuf.Enuf(*args, precision=prec, force_mode=mode)
    d = _eval(ref, xt, qt, torch.cuda.current_stream())
    tol = 1e-12 if prec == "f64" else 1e-5
    assert abs(d[0][0] - a[0][0]) <= tol * np.abs(a[0][1:]).sum()
    for k in range(1, 5):
        assert rms_rel(d[k], a[k]) <= tol
