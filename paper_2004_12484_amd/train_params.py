"""Train and evaluate the ENUF parameter predictor.

    python -m paper_2004_12484_amd.train_params train --sweeps a.npz b.npz
    python -m paper_2004_12484_amd.train_params evaluate --sweeps a.npz b.npz --out eval.json

train:    labels = the fastest swept setting meeting each target error
          (grid search over the sweep), features from the system; systems
          whose seed is a multiple of 10 are held out.  The network is trained
          with the library's MLP kernels and saved to data/param_mlp.npz.
evaluate: for held-out systems and each target, runs ENUF (FP32) with the
          network's setting, the grid-search setting and the Eq. 31-32
          heuristic, measuring error against a tight FP64 reference and GPU
          time; reports success rates and times, including the cost of the
          search itself.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import params as P
from .sweep import combine, system_for_seed

TARGETS = (1e-3, 3e-4, 1e-4, 3e-5)
Y_WEIGHTS = np.array([1.0, 1.0, 1.0, 1.0, 0.5, 1.0], np.float32)


def load_sweeps(paths):
    recs = []
    for path in paths:
        d = np.load(path)
        S, R = d["systems"], d["rows"]
        for i in range(S.shape[0]):
            seed, N, Lx, Ly, Lz, fq, a, cost = S[i]
            recs.append({"seed": int(seed), "N": int(N), "box": np.array([Lx, Ly, Lz]), "f_q": fq, "a": a,
                         "cost_ms": cost, "rows": R[R[:, 0] == i][:, 1:]})
    return recs


def dataset(recs):
    X, Y, meta = [], [], []
    for r in recs:
        settings = combine(r)
        for tgt in TARGETS:
            best = P.grid_search({"settings": settings}, tgt)
            if best is None:
                continue
            X.append(P.features(r["N"], r["box"], r["f_q"], tgt))
            a = r["a"]
            Y.append([best["alpha"] * a, *[math.log2(m) for m in best["M"]], best["p"], best["r_c"] / a])
            meta.append((r["seed"], tgt, best["time"], best["err"], r["cost_ms"]))
    return np.array(X), np.array(Y), meta


def train(paths, epochs=300, seed=0, log=print):
    from .mlp import MLP

    recs = load_sweeps(paths)
    X, Y, meta = dataset(recs)
    held = np.array([m[0] % 10 == 0 for m in meta])
    Xtr, Ytr = X[~held], Y[~held]
    xm, xs = Xtr.mean(0), Xtr.std(0) + 1e-9
    ym, ys = Ytr.mean(0), Ytr.std(0) + 1e-9
    net = MLP(5, 64, 3, 6, seed=seed)
    t0 = time.time()
    hist = net.fit((Xtr - xm) / xs, (Ytr - ym) / ys, Y_WEIGHTS, epochs=epochs, batch=256, lr=3e-3, log=log)
    log(f"trained on {len(Xtr)} samples ({held.sum()} held out) in {time.time() - t0:.1f}s, "
        f"final loss {hist[-1]:.4e}")
    os.makedirs(os.path.dirname(P.MODEL_PATH), exist_ok=True)
    np.savez(P.MODEL_PATH, params=net.numpy_params(), x_mean=xm, x_std=xs, y_mean=ym, y_std=ys,
             dims=np.array([5, 64, 3, 6]), loss=np.array(hist), n_train=len(Xtr))
    P.export_bin(P.MODEL_PATH)
    return hist


def evaluate(paths, out, max_systems=200, log=print):
    import torch

    from . import enuf, inputs
    from .sweep import reference_setting

    held = [r for r in load_sweeps(paths) if r["seed"] % 10 == 0]
    # every held-out large system, then the others spread evenly over the rest
    big = [r for r in held if r["N"] > 262144]
    rest = [r for r in held if r["N"] <= 262144]
    k = max(0, max_systems - len(big))
    stride = max(1, len(rest) // max(1, k))
    recs = big[:max_systems] + rest[::stride][:k]
    pred = P.Predictor()
    dev = torch.device("cuda", 0)
    results = []
    for r in recs:
        w = system_for_seed(r["seed"])
        box = np.asarray(w.box, float)
        x64 = torch.tensor(w.x, dtype=torch.float64, device=dev)
        q64 = torch.tensor(w.q, dtype=torch.float64, device=dev)
        x32, q32 = x64.float(), q64.float()
        charged = torch.tensor(w.q != 0, device=dev)
        ref = reference_setting(w.N, box)
        eng = enuf.Enuf(box, w.N, ref["alpha"], ref["r_c"], ref["M"], ref["p"], precision="f64")
        _, Fref, _ = eng.energy_forces(x64, q64)
        eng.close()
        Fr = Fref[charged]
        nr = torch.linalg.norm(Fr)
        settings = combine(r)

        def run(s):
            if s is None:
                return None
            e = enuf.Enuf(box, w.N, s["alpha"], s["r_c"], s["M"], s["p"], precision="f32")
            e.energy_forces(x32, q32)
            e.set_option(enuf.OPT_TIMING, 3)
            for _ in range(3):
                _, F, _ = e.energy_forces(x32, q32)
            t = sum(e.timings().values())
            e.close()
            return {"err": float((torch.linalg.norm(F.double()[charged] - Fr) / nr).item()), "time_ms": t,
                    "setting": {k: (list(v) if isinstance(v, tuple) else v) for k, v in s.items()
                                if k in ("alpha", "r_c", "M", "p")}}

        for tgt in TARGETS:
            t0 = time.perf_counter()
            sm = pred.select(w.N, box, r["f_q"], tgt)
            t_inf = (time.perf_counter() - t0) * 1e3
            sg = P.grid_search({"settings": settings}, tgt)
            sh = P.heuristic(w.N, box, r["f_q"], tgt)
            results.append({"seed": r["seed"], "N": w.N, "target": tgt, "search_cost_ms": r["cost_ms"],
                            "mlp": run(sm), "mlp_inference_ms": t_inf, "grid": run(sg), "heuristic": run(sh)})
        if len(results) % 40 == 0:
            log(f"[eval] {len(results)} cases")
    summ = {}
    for tgt in TARGETS:
        rs = [x for x in results if x["target"] == tgt and x["grid"] is not None]
        if not rs:
            continue
        def rate(k):
            return float(np.mean([x[k] is not None and x[k]["err"] <= tgt for x in rs]))
        def med_ratio(k):
            v = [x[k]["time_ms"] / x["grid"]["time_ms"] for x in rs if x[k] is not None and x[k]["err"] <= tgt]
            return float(np.median(v)) if v else None
        summ[str(tgt)] = {"cases": len(rs), "mlp_meets_target": rate("mlp"), "heuristic_meets_target": rate("heuristic"),
                          "grid_meets_target": rate("grid"),
                          "mlp_time_over_grid_median": med_ratio("mlp"),
                          "heuristic_time_over_grid_median": med_ratio("heuristic"),
                          "median_search_cost_ms": float(np.median([x["search_cost_ms"] for x in rs])),
                          "median_grid_time_ms": float(np.median([x["grid"]["time_ms"] for x in rs])),
                          "median_mlp_time_ms": float(np.median([x["mlp"]["time_ms"] for x in rs]))}
    by_size = []
    for lo, hi in ((0, 2e4), (2e4, 262144.5), (262144.5, 4.3e6)):
        for tgt in TARGETS:
            rs = [x for x in results if x["target"] == tgt and x["grid"] is not None and lo <= x["N"] < hi]
            if not rs:
                continue
            def ok(k):
                return [x for x in rs if x[k] is not None and x[k]["err"] <= tgt]
            def ratio(k):
                v = [x[k]["time_ms"] / x["grid"]["time_ms"] for x in ok(k)]
                return float(np.median(v)) if v else None
            by_size.append({"N_range": [lo, hi], "target": tgt, "cases": len(rs),
                            "mlp_meets_target": len(ok("mlp")) / len(rs),
                            "heuristic_meets_target": len(ok("heuristic")) / len(rs),
                            "mlp_time_over_grid_median": ratio("mlp"),
                            "heuristic_time_over_grid_median": ratio("heuristic")})
    with open(out, "w") as f:
        json.dump({"summary": summ, "by_size": by_size, "cases": results}, f)
    log(json.dumps(by_size, indent=1))
    log(json.dumps(summ, indent=1))
    return summ


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--sweeps", nargs="+", required=True)
    ap.add_argument("--out", default="param_eval.json")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--max-systems", type=int, default=200)
    args = ap.parse_args(argv)
    if args.cmd == "train":
        train(args.sweeps, epochs=args.epochs, log=lambda s: print(s, flush=True))
    else:
        evaluate(args.sweeps, args.out, args.max_systems, log=lambda s: print(s, flush=True))


if __name__ == "__main__":
    main()
