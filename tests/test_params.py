"""CPU checks of the parameter-selection host logic: the Eq. 31-32 heuristic
reproduces the paper's relations, snapped settings are always valid for
enuf_create, and the separable sweep combination picks consistent rows."""
import math

import numpy as np
import pytest

from paper_2004_12484_amd import params as P
from paper_2004_12484_amd.sweep import combine


def _valid(s, box):
    M = s["M"]
    assert all(8 <= m <= 512 and (m & (m - 1)) == 0 for m in M)
    assert s["p"] in (2, 4, 6, 8) and all(2 * s["p"] <= m for m in M)
    assert 0 < s["r_c"] <= 0.5 * min(box) + 1e-12
    assert s["alpha"] > 0


@pytest.mark.parametrize("target", [1e-3, 1e-4, 1e-5])
def test_heuristic_follows_eq31_32(target):
    box = np.array([30.0, 30.0, 60.0])
    N = 20000
    s = P.heuristic(N, box, 0.5, target)
    _valid(s, box)
    sq = math.sqrt(-math.log(target))
    # Eq. 32 at equality: alpha r_c = sqrt(-ln delta)
    assert abs(s["alpha"] * s["r_c"] - sq) < 1e-12 * sq
    # Eq. 31: the kept modes reach n_c = alpha L sqrt(-ln delta)/pi
    n_c = s["alpha"] * box[0] * sq / math.pi
    assert s["M"][0] >= 2 * round(n_c)
    assert s["M"][2] >= s["M"][0]  # the long axis gets at least as many points


def test_heuristic_paper_worked_numbers():
    # delta = 1e-4 with r_c = 3 R_c (R_c = 1.125 * 6.954 A) implies
    # alpha >= sqrt(-ln 1e-4) / r_c ~ 0.13 A^-1, quoted as alpha >= 0.12 A^-1
    rc = 3.0 * 1.125 * 6.954
    alpha_min = math.sqrt(-math.log(1e-4)) / rc
    assert 0.12 <= alpha_min <= 0.135
    assert math.erfc(0.12 * rc) < 2e-4


@pytest.mark.parametrize("seed", range(5))
def test_snap_gives_valid_settings(seed):
    rng = np.random.default_rng(seed)
    box = np.array([10.0, 10.0, 20.0]) * rng.uniform(0.5, 5)
    s = P.snap(box, 5000, rng.uniform(0.3, 2), rng.uniform(2, 10, 3), rng.uniform(1, 9), rng.uniform(1, 20))
    _valid(s, box)


def test_features_layout():
    f = P.features(1000, [2.0, 3.0, 4.0], 0.25, 1e-4)
    assert np.allclose(f, [3.0, 1.5, 2.0, 0.25, -4.0])


def test_combine_separable_rows():
    # two alphas; kind 0 rows (real-space) x kind 1 rows (reciprocal)
    rows = np.array([
        # alpha, rc, Mx, My, Mz, p, err, time, pair, kind
        [1.0, 3.0, 64, 64, 64, 8, 3e-4, 5.0, 2.0, 0],
        [1.0, 4.2, 32, 32, 32, 4, 4e-4, 3.0, 1.5, 1],
        [2.0, 1.5, 64, 64, 64, 8, 1e-4, 5.0, 1.0, 0],
        [2.0, 2.1, 64, 64, 64, 6, 1e-5, 6.0, 1.0, 1],
    ])
    s = combine({"rows": rows})
    assert len(s) == 2
    a = [x for x in s if x["alpha"] == 1.0][0]
    assert a["M"] == (32, 32, 32) and a["p"] == 4 and a["r_c"] == 3.0
    assert math.isclose(a["err"], 5e-4)
    assert math.isclose(a["time"], 2.0 + 1.5)
    best = P.grid_search({"settings": s}, 2e-4)
    assert best is not None and best["alpha"] == 2.0
    assert P.grid_search({"settings": s}, 1e-6) is None


def test_select_params_rejects_bad_arguments():
    from paper_2004_12484_amd import enuf

    box = [20.0, 20.0, 20.0]
    for args in ((1, box, 0.5, 1e-4), (1000, box, 0.0, 1e-4), (1000, box, 0.5, 0.0), (1000, [20, -1, 20], 0.5, 1e-4)):
        with pytest.raises(enuf.EnufError) as ei:
            P.select_params(*args)
        assert ei.value.status == enuf.ENUF_EINVAL


def test_select_params_network_file_checks(tmp_path):
    """A malformed network file is refused; a valid one is not evaluated for
    a system outside its training ranges (the heuristic is used, no GPU)."""
    from paper_2004_12484_amd import enuf

    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTANET!" + b"\0" * 64)
    with pytest.raises(enuf.EnufError) as ei:
        P.select_params(5000, [20.0, 20.0, 20.0], 0.5, 1e-4, model_path=str(bad))
    assert ei.value.status == enuf.ENUF_EINVAL
    with pytest.raises(enuf.EnufError):
        P.select_params(5000, [20.0, 20.0, 20.0], 0.5, 1e-4, model_path=str(tmp_path / "missing.bin"))
    good = P.export_bin(P.MODEL_PATH, out=str(tmp_path / "net.bin"))
    box = [200.0, 200.0, 200.0]
    N = 20_000_000   # above the training range
    s, method = P.select_params(N, box, 0.5, 1e-4, model_path=good)
    assert method == "heuristic"
    assert s == P.heuristic(N, box, 0.5, 1e-4)
    # a 1:2:1 box is not a trained shape (the network saw 1:1:1 and 1:1:2)
    assert not P.in_training_range(20000, [20.0, 40.0, 20.0], 0.5, 1e-4)
    assert P.in_training_range(20000, [20.0, 20.0, 40.0], 0.5, 1e-4)
