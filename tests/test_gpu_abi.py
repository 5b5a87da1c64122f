"""GPU checks of the C ABI's workspace and replay calls.

* A context has no device memory until a workspace is given: evaluating
  before that is a call-sequence error; a workspace smaller than
  enuf_workspace_bytes() is rejected; a library-allocated workspace gives
  the same results as a caller-owned one.
* Graph replay (ENUF_OPT_GRAPH) gives the results of the launched sequence
  on every replay, with eager work and synchronisations between replays, and
  captures again when the arguments or options change.
* The copy probe copies exactly and rejects bad arguments.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import enuf_mirror as em  # noqa: E402
from paper_2004_12484_amd import enuf  # noqa: E402

from gpu_util import rms_rel, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _sys(n=600, box=(9.0, 10.0, 11.0), seed=31):
    rng = np.random.default_rng(seed)
    box = np.asarray(box, float)
    x = rng.uniform(0, 1, (n, 3)) * box
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0) * rng.uniform(0.5, 1.5, n)
    return x, q, box


ARGS = (1.1, 4.0, (32, 32, 32), 4)


def test_evaluation_without_workspace_is_state_error():
    x, q, box = _sys()
    eng = enuf.Enuf(box, len(q), *ARGS, workspace=False)
    with pytest.raises(enuf.EnufError) as ei:
        eng.energy_forces(to_dev(x, torch.float64), to_dev(q, torch.float64))
    assert ei.value.status == enuf.ENUF_ESTATE


def test_workspace_too_small_is_rejected():
    x, q, box = _sys()
    eng = enuf.Enuf(box, len(q), *ARGS, workspace=False)
    lib = enuf.load_library()
    nb = ctypes.c_size_t()
    assert lib.enuf_workspace_bytes(eng._h, ctypes.byref(nb)) == 0
    buf = torch.empty(nb.value - 512, dtype=torch.uint8, device="cuda")
    assert lib.enuf_set_workspace(eng._h, enuf._ptr(buf), buf.numel()) == enuf.ENUF_EINVAL
    assert b"too small" in lib.enuf_last_error(eng._h)
    assert lib.enuf_set_workspace(eng._h, None, nb.value) == enuf.ENUF_EINVAL


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_library_workspace_matches_caller_workspace(prec):
    x, q, box = _sys(seed=32)
    a = enuf.Enuf(box, len(q), *ARGS, precision=prec)
    b = enuf.Enuf(box, len(q), *ARGS, precision=prec, workspace=False)
    lib = enuf.load_library()
    b._bind_stream()
    assert lib.enuf_alloc_workspace(b._h) == 0
    dt = a.dtype
    Ea, Fa, pa = a.energy_forces(to_dev(x, dt), to_dev(q, dt), potential=True)
    Eb, Fb, pb = b.energy_forces(to_dev(x, dt), to_dev(q, dt), potential=True)
    tol = 1e-12 if prec == "f64" else 1e-6
    assert float((Ea - Eb).abs().max()) <= tol * float(Ea.abs().max())
    assert rms_rel(Fb.double().cpu().numpy(), Fa.double().cpu().numpy()) <= tol
    assert rms_rel(pb.double().cpu().numpy(), pa.double().cpu().numpy()) <= tol
    # a second workspace set on the same context forgets the evaluation
    ws2 = torch.empty_like(a._ws)
    a._bind_stream()
    assert lib.enuf_set_workspace(a._h, enuf._ptr(ws2), ws2.numel()) == 0
    with pytest.raises(enuf.EnufError):
        a.energy_grad(1.0)
    a._ws = ws2
    Ec, Fc, _ = a.energy_forces(to_dev(x, dt), to_dev(q, dt), potential=True)
    assert float((Ea - Ec).abs().max()) <= tol * float(Ea.abs().max())


@pytest.mark.parametrize("mode", ["ik", "analytic"])
def test_graph_replay_matches_launched_sequence(mode):
    x, q, box = _sys(n=900, seed=33)
    eng = enuf.Enuf(box, len(q), *ARGS, force_mode=mode)
    xt, qt = to_dev(x, torch.float64), to_dev(q, torch.float64)
    E0, F0, p0 = eng.energy_forces(xt, qt, potential=True)
    E0, F0, p0 = E0.clone(), F0.clone(), p0.clone()
    eng.set_option(enuf.OPT_GRAPH, 1)
    E = torch.empty(5, dtype=torch.float64, device="cuda")
    F = torch.empty((len(q), 3), dtype=torch.float64, device="cuda")
    phi = torch.empty(len(q), dtype=torch.float64, device="cuda")
    lib = enuf.load_library()
    for rep in range(4):
        # eager work between replays, on the same stream
        F.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64).sum()
        assert lib.enuf_energy_forces(eng._h, enuf._ptr(xt), enuf._ptr(qt), enuf._ptr(E), enuf._ptr(F),
                                      enuf._ptr(phi)) == 0
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert float((E - E0).abs().max()) <= 1e-12 * float(E0.abs().max()), rep
        assert rms_rel(F.cpu().numpy(), F0.cpu().numpy()) <= 1e-12, rep
        assert rms_rel(phi.cpu().numpy(), p0.cpu().numpy()) <= 1e-12, rep
    # new positions in a new tensor: captured again, and the results follow
    x2 = x + 0.05
    xt2 = to_dev(x2, torch.float64)
    assert lib.enuf_energy_forces(eng._h, enuf._ptr(xt2), enuf._ptr(qt), enuf._ptr(E), enuf._ptr(F),
                                  enuf._ptr(phi)) == 0
    torch.cuda.synchronize()
    m = em.enuf(x2, q, box, *ARGS, want_grad=mode == "analytic")
    Fref = m["F"] if mode == "ik" else -m["grad_x"]
    assert rms_rel(F.cpu().numpy(), Fref) <= 1e-10
    # an option change (ke = 2) is captured again too
    eng.set_option(enuf.OPT_KE, 2.0)
    assert lib.enuf_energy_forces(eng._h, enuf._ptr(xt2), enuf._ptr(qt), enuf._ptr(E), enuf._ptr(F),
                                  enuf._ptr(phi)) == 0
    torch.cuda.synchronize()
    assert rms_rel(F.cpu().numpy(), 2.0 * Fref) <= 1e-10
    # the adjoint reads the graph evaluation's state
    gx, gq = eng.energy_grad(1.0)
    assert rms_rel(gq.cpu().numpy(), 2.0 * m["phi"]) <= 1e-10
    # per-phase timing is not recorded in graph mode
    eng.set_option(enuf.OPT_TIMING, 4)
    with pytest.raises(enuf.EnufError):
        eng.timings()


def test_copy_probe_copies_and_validates():
    """enuf_copy_probe (the bandwidth probe): an exact copy of sizes that do
    and do not fill the kernel's four-deep loop, and the argument checks."""
    lib = enuf.load_library()
    for nbytes in (16, 16 * 1000 + 16 * 7, 3 << 20):
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
        dst = torch.zeros_like(src)
        enuf.copy_probe(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
    src = torch.zeros(64, dtype=torch.uint8, device="cuda")
    dst = torch.zeros(64, dtype=torch.uint8, device="cuda")
    vp = ctypes.c_void_p
    assert lib.enuf_copy_probe(vp(src.data_ptr()), vp(dst.data_ptr()), 20, None) == enuf.ENUF_EINVAL
    assert lib.enuf_copy_probe(vp(src.data_ptr() + 4), vp(dst.data_ptr()), 16, None) == enuf.ENUF_EINVAL
    assert lib.enuf_copy_probe(None, vp(dst.data_ptr()), 16, None) == enuf.ENUF_EINVAL
    assert lib.enuf_copy_probe(vp(src.data_ptr()), vp(src.data_ptr() + 16), 32, None) == enuf.ENUF_EINVAL
