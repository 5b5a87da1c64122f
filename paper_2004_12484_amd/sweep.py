"""Error/time sweeps of ENUF on random neutral systems (training data for the
parameter predictor).

    python -m paper_2004_12484_amd.sweep --seeds 1000:3000 --out sweep.npz

For each seeded system (inputs.random_system):
  * a tight FP64 reference: alpha_ref r_c,ref = 4.2 (erfc ~ 3e-9), grid with
    alpha_ref h <= 0.35 and p = 8, so that its forces are the converged Ewald
    forces to ~1e-7;
  * the real-space truncation error eps_R(alpha, r_c): FP32 evaluations with
    the reciprocal part converged (alpha h <= 0.35, p = 8);
  * the reciprocal error eps_K(alpha, M, p): FP32 evaluations with the real
    part converged (alpha r_c = 4.2);
  * GPU time of the pair phase and of everything else, from the library's
    per-phase HIP events.
Errors are RMS relative force errors over the charged particles.  The error
of a full setting is taken as sqrt(eps_R^2 + eps_K^2) and its time as
t_pair(alpha, r_c) + t_rest(alpha, M, p); the two parts are independent sums.
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import numpy as np
import torch

from . import enuf, inputs
from .params import M_MIN, spacing

ALPHA_A = (0.7, 0.95, 1.2)          # alpha in units of 1/a
ALPHA_RC = (2.5, 3.0, 3.5)          # alpha * r_c
ALPHA_H = (0.45, 0.6, 0.8)          # alpha * grid spacing
P_SET = (4, 6, 8)
ALPHA_RC_CONV = 4.2
ALPHA_H_CONV = 0.35


SWEEP_M_MAX = 1024  # the library's largest grid: large systems need it for the tight reference


def pow2_ceil(v):
    return int(min(SWEEP_M_MAX, max(M_MIN, 2 ** math.ceil(math.log2(max(v, 1.0))))))


def grid_for(alpha, box, ah):
    return tuple(pow2_ceil(alpha * float(L) / ah) for L in box)


def _run(x, q, box, alpha, rc, M, p, prec, reps=2):
    eng = enuf.Enuf(box, len(q), alpha, rc, M, p, precision=prec)
    E, F, _ = eng.energy_forces(x, q)
    eng.set_option(enuf.OPT_TIMING, 1)
    best = None
    for _ in range(reps):
        E, F, _ = eng.energy_forces(x, q)
        ph = eng.timings()
        tot = sum(ph.values())
        if best is None or tot < best[0]:
            best = (tot, ph["pair"])
    eng.close()
    return F, best[0], best[1]


def reference_setting(N, box):
    """The tight FP64 setting the sweep errors are measured against:
    alpha r_c = 4.2 (erfc ~ 3e-9), alpha h <= 0.35, p = 8."""
    box = np.asarray(box, float)
    a = spacing(N, box)
    rc_ref = min(0.499 * float(box.min()), 3.5 * a)
    alpha_ref = ALPHA_RC_CONV / rc_ref
    return {"alpha": alpha_ref, "r_c": rc_ref, "M": grid_for(alpha_ref, box, ALPHA_H_CONV), "p": 8}


def sweep_arrays(x, q, box):
    """The separable sweep of one system given as arrays (positions [N,3],
    charges [N], box [3]); returns the record `combine` takes."""
    box = np.asarray(box, float)
    q = np.asarray(q, float)
    N = len(q)
    a = spacing(N, box)
    lmin = float(box.min())
    dev = torch.device("cuda", 0)
    x64 = torch.tensor(np.asarray(x, float), dtype=torch.float64, device=dev)
    q64 = torch.tensor(q, dtype=torch.float64, device=dev)
    x32 = x64.float()
    q32 = q64.float()
    charged = torch.tensor(q != 0, device=dev)
    ref = reference_setting(N, box)
    F_ref, t_ref, _ = _run(x64, q64, box, ref["alpha"], ref["r_c"], ref["M"], ref["p"], "f64", reps=1)
    Fr = F_ref[charged]
    nref = torch.linalg.norm(Fr)
    del F_ref

    def err(F):
        return float((torch.linalg.norm(F.double()[charged] - Fr) / nref).item())

    rows = []
    cost = t_ref
    for aa in ALPHA_A:
        alpha = aa / a
        rc_conv = ALPHA_RC_CONV / alpha
        if rc_conv > 0.499 * lmin:
            continue
        M_conv = grid_for(alpha, box, ALPHA_H_CONV)
        for arc in ALPHA_RC:
            rc = arc / alpha
            F, t, tp = _run(x32, q32, box, alpha, rc, M_conv, 8, "f32")
            rows.append((alpha, rc, *M_conv, 8, err(F), t, tp, 0))
            cost += t
        seen = set()
        for ah in ALPHA_H:
            M = grid_for(alpha, box, ah)
            for p in P_SET:
                if any(2 * p > m for m in M) or (M, p) in seen:
                    continue
                seen.add((M, p))
                F, t, tp = _run(x32, q32, box, alpha, rc_conv, M, p, "f32")
                rows.append((alpha, rc_conv, *M, p, err(F), t, tp, 1))
                cost += t
    return {"N": N, "box": box, "f_q": float(np.count_nonzero(q)) / N, "a": a,
            "rows": np.array(rows, float).reshape(-1, 10), "cost_ms": cost}


# the system families of the training data: seeds below LARGE_SEED0 are the
# small and medium systems; then the large ones (up to the 4M-site workload,
# charged fractions down to 0.02); from DENSE_SEED0 large dense and mostly
# charged ones (the one-million-ion regime)
LARGE_SEED0 = 5000
LARGE = dict(n_min=262144, n_max=4194304, fq_min=0.02)
DENSE_SEED0 = 5400
DENSE = dict(n_min=262144, n_max=2097152, fq_min=0.5, rho_min=1.0, rho_max=3.15)


def system_for_seed(seed):
    if seed >= DENSE_SEED0:
        return inputs.random_system(seed, **DENSE)
    if seed >= LARGE_SEED0:
        return inputs.random_system(seed, **LARGE)
    return inputs.random_system(seed)


def sweep_system(seed):
    w = system_for_seed(seed)
    rec = sweep_arrays(w.x, w.q, w.box)
    rec["seed"] = seed
    return rec


def combine(rec):
    """Full settings from one system's separable sweep: every (alpha, r_c)
    row of kind 0 with every (alpha, M, p) row of kind 1 at the same alpha."""
    # columns: alpha, r_c, Mx, My, Mz, p, err, time, pair time, kind
    rows = rec["rows"]
    out = []
    for ra in rows[rows[:, 9] == 0]:
        for rb in rows[rows[:, 9] == 1]:
            if abs(ra[0] - rb[0]) > 1e-12 * ra[0]:
                continue
            e = math.hypot(ra[6], rb[6])
            t = ra[8] + (rb[7] - rb[8])  # pair of the first + the rest of the second
            out.append({"alpha": ra[0], "r_c": ra[1], "M": tuple(int(v) for v in rb[2:5]), "p": int(rb[5]),
                        "err": e, "time": t})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", default="1000:1010")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    s0, s1 = (int(v) for v in args.seeds.split(":"))
    recs = []
    t0 = last = time.time()
    for k, seed in enumerate(range(s0, s1)):
        recs.append(sweep_system(seed))
        if k % 50 == 0 or seed == s1 - 1 or time.time() - last > 30:
            last = time.time()
            print(f"[sweep] seed {seed} N={recs[-1]['N']} rows={len(recs[-1]['rows'])} "
                  f"elapsed {last - t0:.0f}s", flush=True)
    sys_arr = np.array([[r["seed"], r["N"], *r["box"], r["f_q"], r["a"], r["cost_ms"]] for r in recs], float)
    rows = np.concatenate([np.column_stack([np.full(len(r["rows"]), i), r["rows"]]) for i, r in enumerate(recs)])
    np.savez_compressed(args.out, systems=sys_arr, rows=rows,
                        columns=np.array(["sys", "alpha", "r_c", "Mx", "My", "Mz", "p", "err", "time_ms",
                                          "pair_ms", "kind"]))
    print(f"[sweep] wrote {args.out}: {len(recs)} systems, {len(rows)} evaluations", flush=True)


if __name__ == "__main__":
    main()
