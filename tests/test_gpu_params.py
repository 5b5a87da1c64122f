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
