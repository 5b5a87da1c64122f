"""Host-side checks of the benchmark's bookkeeping (no GPU)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _W:
    M = (256, 256, 256)


def test_algorithmic_bytes_follow_the_field_count():
    G = 256 ** 3
    # analytic forces: one potential spectrum back, a scalar real grid
    a = bench.algorithmic_bytes(_W, 4, 1 << 20, nfield=1, out_reals=1)
    assert a["influence_z"] == 2 * G * 4
    assert a["fft_inv"] == 4 * G * 4          # y read+write, x read, x write
    assert a["gather"] == (1 << 20) * (16 + 4 + 12) + G * 4
    # ik forces with potentials: four spectra, an interleaved real4 grid
    b = bench.algorithmic_bytes(_W, 4, 1 << 20, nfield=4, out_reals=4)
    assert b["influence_z"] == 5 * G * 4
    assert b["fft_inv"] == (8 + 4 + 4) * G * 4
    assert b["gather"] - a["gather"] == 3 * G * 4
    assert a["spread"] == b["spread"] and a["fft_fwd"] == b["fft_fwd"] == 4 * G * 4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_pair_count_is_unordered_pairs_of_a_uniform_fluid():
    # count the unordered pairs inside r_c of a seeded uniform system (the
    # one-million-ion density) directly, with periodic images
    from scipy.spatial import cKDTree

    L, rc, n = 17.5, 1.8, 16384
    x = np.random.default_rng(0).uniform(0.0, L, (n, 3))
    pairs = len(cKDTree(x, boxsize=L).query_pairs(rc))
    w = type("W", (), {"box": np.array([L, L, L]), "r_c": rc})
    est = bench.pair_count(w, n)
    # Poisson-like scatter of ~600k pairs: well under 1%
    assert abs(est - pairs) <= 0.01 * pairs, (est, pairs)
