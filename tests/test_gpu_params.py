"""GPU checks of the parameter selection: the sweep's tight FP64 reference
against the oracle, and the trained network against the oracle and against
the Eq. 31-32 heuristic.

The systems are fresh random neutral systems (seeds below the sweep's range,
1000 <= N <= 3000 so that the oracle finishes in seconds), never seen in training.
The oracle reference is the converged Ewald force at a splitting of its own
choosing (the converged force does not depend on alpha): alpha r_c = 5.5 at
r_c = min(L)/2 and every k with exp(-k^2/4 alpha^2) >= 1e-14.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ewald as ew  # noqa: E402
from paper_2004_12484_amd import inputs  # noqa: E402
from paper_2004_12484_amd import params as P  # noqa: E402
from paper_2004_12484_amd.sweep import reference_setting  # noqa: E402

from gpu_util import rms_rel, run  # noqa: E402

pytestmark = pytest.mark.gpu


def _systems(seeds):
    return [inputs.random_system(s, n_min=1000, n_max=3000) for s in seeds]


def _oracle_forces(w):
    rc = 0.5 * float(np.min(w.box))
    alpha = 5.5 / rc
    r = ew.ewald(w.x, w.q, w.box, alpha, rc, tol=1e-14)
    return r["F"]


def _err(F, Fo, q):
    c = q != 0
    return rms_rel(F[c], Fo[c])


def test_sweep_reference_matches_oracle():
    # the error labels of the training sweeps are measured against this
    # reference; it must sit far below the smallest target (3e-5)
    errs = []
    for w in _systems(range(100, 120)):
        ref = reference_setting(w.N, w.box)
        _, out = run(w.x, w.q, w.box, ref["alpha"], ref["r_c"], ref["M"], ref["p"], precision="f64",
                     potential=False)
        errs.append(_err(out["F"], _oracle_forces(w), w.q))
    print("sweep reference eps_F: max %.2e median %.2e" % (max(errs), float(np.median(errs))))
    assert max(errs) <= 1e-6


@pytest.mark.skipif(not os.path.exists(P.MODEL_PATH), reason="trained parameter model not present")
def test_library_selection_equals_network_prediction():
    """enuf_select_params with the network file gives the network's own
    prediction (forward kernel through the Python binding), snapped."""
    pred = P.Predictor()
    rng = np.random.default_rng(7)
    for k in range(40):
        w = inputs.random_system(300 + k)
        fq = float(np.count_nonzero(w.q)) / w.N
        tgt = float(10 ** rng.uniform(-4.5, -3))
        s, method = P.select_params(w.N, w.box, fq, tgt, model_path=P.MODEL_BIN)
        assert method == "network"
        y = pred.predict_raw(P.features(w.N, w.box, fq, tgt))[0]
        ref = P.snap(w.box, w.N, y[0], y[1:4], y[4], y[5])
        assert s["M"] == ref["M"] and s["p"] == ref["p"], (s, ref)
        assert abs(s["alpha"] - ref["alpha"]) <= 1e-6 * ref["alpha"]
        assert abs(s["r_c"] - ref["r_c"]) <= 1e-6 * ref["r_c"]


@pytest.mark.skipif(not os.path.exists(P.MODEL_PATH), reason="trained parameter model not present")
def test_trained_network_meets_targets_on_fresh_systems():
    pred = P.Predictor()
    hits = {1e-3: 0, 1e-4: 0}
    systems = _systems(range(200, 220))
    for w in systems:
        Fo = _oracle_forces(w)
        fq = float(np.count_nonzero(w.q)) / w.N
        for tgt in hits:
            s = pred.select(w.N, w.box, fq, tgt)
            _, out = run(w.x, w.q, w.box, s["alpha"], s["r_c"], s["M"], s["p"], precision="f32",
                         potential=False)
            e = _err(out["F"], Fo, w.q)
            hits[tgt] += e <= tgt
    rates = {t: h / len(systems) for t, h in hits.items()}
    print("network success rates:", rates)
    assert rates[1e-3] >= 0.9
    assert rates[1e-4] >= 0.8


def _time_and_error(w, s, Fr, charged, x32, q32, reps=5):
    from paper_2004_12484_amd import enuf

    eng = enuf.Enuf(w.box, w.N, s["alpha"], s["r_c"], s["M"], s["p"], precision="f32")
    eng.energy_forces(x32, q32)
    eng.set_option(enuf.OPT_TIMING, reps)
    for _ in range(reps):
        _, F, _ = eng.energy_forces(x32, q32)
    t = sum(eng.timings().values())
    err = float((torch.linalg.norm(F.double()[charged] - Fr) / torch.linalg.norm(Fr)).item())
    eng.close()
    return t, err


@pytest.mark.skipif(not os.path.exists(P.MODEL_PATH), reason="trained parameter model not present")
def test_network_beats_heuristic_time_to_target():
    """What the trained network gains over the method without it: on fresh
    systems (30k .. 300k particles, seeds outside the training sets), at the
    force targets 1e-3 and 3e-4, the network's setting reaches the target in
    less GPU time than the Eq. 31-32 heuristic's, at the median, and meets
    it as often.  A system whose FP32 floor (the FP32 form at the tight
    reference setting, set by position rounding in large dilute boxes) is
    above a third of a target cannot meet it with any parameters; such
    (system, target) cases are left out."""
    from paper_2004_12484_amd import enuf

    ratios, hits_net, hits_heu, used = [], 0, 0, 0
    for seed in range(9000, 9012):
        w = inputs.random_system(seed, n_min=30000, n_max=300000)
        fq = float(np.count_nonzero(w.q)) / w.N
        x64 = torch.tensor(w.x, dtype=torch.float64, device="cuda")
        q64 = torch.tensor(w.q, dtype=torch.float64, device="cuda")
        charged = torch.tensor(w.q != 0, device="cuda")
        ref = reference_setting(w.N, w.box)
        eng = enuf.Enuf(w.box, w.N, ref["alpha"], ref["r_c"], ref["M"], ref["p"], precision="f64")
        _, Fref, _ = eng.energy_forces(x64, q64)
        Fr = Fref[charged]
        eng.close()
        _, floor = _time_and_error(w, ref, Fr, charged, x64.float(), q64.float(), reps=1)
        for tgt in (1e-3, 3e-4):
            if floor > tgt / 3:
                continue
            used += 1
            s_net, method = P.select_params(w.N, w.box, fq, tgt, model_path=P.MODEL_BIN)
            assert method == "network"
            s_heu = P.heuristic(w.N, w.box, fq, tgt)
            t_net, e_net = _time_and_error(w, s_net, Fr, charged, x64.float(), q64.float())
            t_heu, e_heu = _time_and_error(w, s_heu, Fr, charged, x64.float(), q64.float())
            hits_net += e_net <= tgt
            hits_heu += e_heu <= tgt
            if e_net <= tgt and e_heu <= tgt:
                ratios.append(t_net / t_heu)
            print(f"seed {seed} N={w.N} f_q={fq:.2f} target {tgt:.0e}: network {t_net:.3f} ms (eps {e_net:.1e}), "
                  f"heuristic {t_heu:.3f} ms (eps {e_heu:.1e})")
    med = float(np.median(ratios))
    print(f"network/heuristic time at equal target: median {med:.3f} over {len(ratios)} cases; "
          f"target met {hits_net}/{used} (network), {hits_heu}/{used} (heuristic)")
    assert used >= 12
    assert hits_net >= hits_heu - 1
    assert hits_net >= 0.9 * used
    assert med < 1.0
