#!/usr/bin/env python
"""ENUF energy+force throughput on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload ions_1m]

One step = one full ENUF evaluation (enuf_energy_forces: wrap and sort,
spread, forward FFT, influence + energy, inverse FFTs, gather, real-space pair
sum, FP64 energy reduction) of a seeded synthetic system whose positions and
charges are already resident in device memory.  Prints one JSON line with the
throughput (evaluations per second, K steps with nothing else on the stream),
the per-phase times measured with HIP events on the library's stream over a
second pass of the same K steps, the roofline figures of the dominant kernel,
the force/energy error against stored oracle values, and the CPU oracle timed
on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "energy+force evals/sec and ns/particle at 1M ions, RMS force err ≤1e-4"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_TFLOPS = 157.3       # MI355X vector FP32
FP64_VALU_TFLOPS = 78.6
PAIR_FLOPS = 40.0              # flops per evaluated pair (erfc, exp, rsqrt, accumulation)

# Bench workloads: one million ions (every bead of the 1M-bead fluid charged,
# at the searched FP32 setting) is the headline; charged_fluid is the same
# geometry with 20% of the beads charged; the others are smaller and larger
# systems.
WORKLOADS = {
    "charged_fluid": dict(gen="charged_fluid", kw=dict(alpha=0.95)),
    "ions_1m": dict(gen="ions_1m", kw={}, force_mode="analytic",
                    # the plain FP64 form's fastest setting with eps_F <= 1e-4
                    # (bench.py --search --precision f64: 3.02 ms, eps_F 4.9e-5)
                    fp64_form=dict(force_mode="analytic", M=(256, 256, 256), p=6, r_c=1.8, alpha=2.9 / 1.8),
                    # the parameter network's own setting for the same target
                    learned_form=1e-4),
    "electrolyte": dict(gen="electrolyte", kw={}),
    "nacl": dict(gen="nacl", kw={}),
    # 4M sites in 120 x 120 x 240: parameters from the selector (the network,
    # or a grid search over a sweep of the system when it lies outside the
    # network's training range) at the FP32 form's accuracy bar 5e-4 (FP32
    # rounding of the positions alone costs ~2.8e-4 here: chain beads come
    # within a few hundredths of each other), forces and dE/dq
    "anisotropic_selected": dict(gen="anisotropic", kw={}, select=5e-4, potential=True, golden="anisotropic"),
    # the same system at the parameter network's setting for 1e-4 (the
    # stated 256 x 256 x 512 grid with p = 6 comes out of it); forces and
    # dE/dq from the potential grid alone (analytic mode: one field instead
    # of four, 1.6x faster at the same error)
    "anisotropic": dict(gen="anisotropic", kw={}, select=1e-4, potential=True, force_mode="analytic"),
    # ... and at the fastest setting of a timed sweep at the stated grid
    # (alpha r_c in 2.6 .. 3.5, r_c in 2.5 .. 4.5; all met 1e-4)
    "anisotropic_swept": dict(gen="anisotropic", kw=dict(alpha=0.8, r_c=4.0, M=(256, 256, 512), p=6),
                              potential=True, golden="anisotropic"),
    # ENUF-DPD: the charged fluid read as a DPD system (R_c = 1, density ~3,
    # real-space cutoff 3 R_c) of Slater-smeared charges with beta = 1.125
    # (decay length 1/1.125)
    "dpd_slater": dict(gen="charged_fluid", kw=dict(alpha=0.95), slater=1.0 / 1.125),
}


def algorithmic_bytes(w, rs, nq, nfield, out_reals):
    """Algorithmic HBM bytes of each HBM-bound phase for one evaluation.

    rs = bytes per real; nq = active (charged) particles; G = grid points (the
    half spectrum, Mx/2 x My x Mz complex, is also G reals); nfield = field
    spectra transformed back (ik: E_x, E_y, E_z and, with potentials, psi;
    analytic: psi alone); out_reals = reals per grid point of the real field
    array the gather reads (ik: 4, interleaved; analytic: 1).
    spread:  read particles (4 reals) + write the grid once
    fft_fwd: x pass read G reals / write G; y pass read + write G
    influence_z: read G, write nfield x G
    fft_inv: y pass read + write nfield x G; x pass read nfield x G, write the
             real field array G x out_reals
    gather:  read particles (4 reals) + perm (4 B) + fields (G x out_reals)
             and write 3 force reals per particle
    """
    G = int(np.prod(w.M))
    return {
        "spread": nq * 4 * rs + G * rs,
        "fft_fwd": 2 * G * rs + 2 * G * rs,
        "influence_z": G * rs + nfield * G * rs,
        "fft_inv": 2 * nfield * G * rs + (nfield * G * rs + out_reals * G * rs),
        "gather": nq * (4 * rs + 4 + 3 * rs) + out_reals * G * rs,
    }


# phase -> kernel of that phase whose counters profiles/traffic_<workload>.json holds
PHASE_KERNEL = {"pair": "k_pair", "gather": "k_gather_tile", "spread": "k_spread_mfma"}


def sources_sha():
    """Hash of the library sources: counter bytes are reported only for the
    build they were measured on."""
    import glob
    import hashlib

    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2004_12484_amd", "csrc", "*"))
                   + glob.glob(os.path.join(ROOT, "include", "*.h")))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, phase):
    """HBM bytes per launch of the phase's kernel from rocprofv3 FETCH_SIZE and
    WRITE_SIZE counters (each scaled by what the counter reads for a plain
    copy of known size), if they were taken on this exact build.  workload is
    the benchmark's workload key: the counters belong to its setting."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path) or phase not in PHASE_KERNEL:
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources_sha") != sources_sha():
        return None
    k = t["kernels"].get(PHASE_KERNEL[phase])
    if k is None:
        return None
    return 1024.0 * (k["fetch_kib"] * t["fetch_scale"] + k["write_kib"] * t["write_scale"])


def pair_count(w, nq):
    """Expected number of unordered charged pairs inside r_c for a uniform
    fluid: N_q n_nb / 2 with n_nb = (N_q / V) (4/3) pi r_c^3 neighbours."""
    V = float(np.prod(w.box))
    return 0.5 * nq * (nq / V) * 4.0 / 3.0 * math.pi * w.r_c ** 3


def cpu_baseline(w, budget_s=20.0):
    """Time the FP64 oracle on a bounded sub-system of the workload and scale
    to the full system by its operation counts (k-space sum linear in the
    charged count, brute-force real-space sum quadratic)."""
    from oracle import ewald as ew

    charged = np.nonzero(w.q)[0]
    nq_full = len(charged)
    n_s = min(nq_full, 2048)
    while True:
        sel = charged[:n_s]
        x, q = w.x[sel], w.q[sel]
        t0 = time.perf_counter()
        ew.real_minimage(x, q, w.box, w.alpha, w.r_c, sample=np.zeros(0, np.int64))
        t_real = time.perf_counter() - t0
        nmax, kc2 = ew.kset_converged(w.box, w.alpha)
        t0 = time.perf_counter()
        ew.recip(x, q, w.box, w.alpha, nmax=nmax, kcut2=kc2, sample=np.zeros(0, np.int64))
        t_rec = time.perf_counter() - t0
        if t_real + t_rec > 2.0 or n_s >= nq_full or n_s >= 65536:
            break
        n_s *= 2
    scale = nq_full / n_s
    t_full = t_rec * scale + t_real * scale * scale
    return {
        "value": 1.0 / t_full, "unit": "evals/s", "cores": ew.num_threads(), "kind": "oracle",
        "sample": (f"direct FP64 Ewald oracle on the first {n_s} charged particles of the workload "
                   f"(same box, alpha, r_c, k-set converged to 1e-16): real space {t_real:.3f} s "
                   f"(scaled x{scale:.1f}^2), k space {t_rec:.3f} s (scaled x{scale:.1f}); "
                   f"extrapolated {t_full:.1f} s per full evaluation"),
    }


def golden_check(w, F, E, phi=None, name=None):
    """RMS relative force error and relative energy error against stored oracle
    values for this workload (tests/golden/<name>_oracle.npz, name defaulting
    to the generator's), if present.  Files holding only F_conv (the converged
    Ewald force, whatever splitting parameter the oracle used) are compared on
    forces alone."""
    path = os.path.join(ROOT, "tests", "golden", f"{name or w.name}_oracle.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path)
    if int(g["N"]) != w.N or int(g["seed"]) != w.seed:
        return None
    s = g["sample"]
    Fs = F[s]
    out = {"force_sample": int(len(s)), "ref_tol": float(g["tol"])}
    if "F" in g.files:
        if not (np.isclose(float(g["alpha"]), w.alpha) and np.isclose(float(g["r_c"]), w.r_c)):
            return None
        out["rms_force_err"] = float(np.linalg.norm(Fs - g["F"]) / np.linalg.norm(g["F"]))
    if "F_conv" in g.files:
        # against the Ewald sum with the real-space cut converged
        out["rms_force_err_rc_converged"] = float(np.linalg.norm(Fs - g["F_conv"]) / np.linalg.norm(g["F_conv"]))
        out.setdefault("rms_force_err", out["rms_force_err_rc_converged"])
    if "E" in g.files and np.isclose(float(g["alpha"]), w.alpha) and np.isclose(float(g["r_c"]), w.r_c):
        out["energy_rel_err"] = float(abs(E - float(g["E"])) / abs(float(g["E"])))
    if "E_table" in g.files:
        # Ewald energy at this (alpha, r_c), stored per setting
        for a, rc, e_ref in g["E_table"]:
            if np.isclose(a, w.alpha) and np.isclose(rc, w.r_c):
                out["energy_rel_err"] = float(abs(E - e_ref) / abs(e_ref))
    if "E_conv" in g.files:
        # against the converged Coulomb energy (alpha-independent)
        out["energy_rel_err_conv"] = float(abs(E - float(g["E_conv"])) / abs(float(g["E_conv"])))
    if phi is not None and ("phi_conv" in g.files or "phi" in g.files):
        # dE/dq against the (converged) potentials
        ref = g["phi_conv"] if "phi_conv" in g.files else g["phi"]
        out["rms_dEdq_err"] = float(np.linalg.norm(phi[s] - ref) / np.linalg.norm(ref))
    return out


def copy_probe(dev, mib=1024, reps=10):
    """Achievable copy bandwidth, the second denominator of the HBM-bound
    kernels: the library's plain copy kernel over 1 GiB (read + write bytes
    per second, HIP events around `reps` copies after two warm-ups)."""
    import torch
    from paper_2004_12484_amd import enuf
    nbytes = mib << 20
    src = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        enuf.copy_probe(src, dst)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        enuf.copy_probe(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes_copied": nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9,
            "kernel": "enuf_copy_probe (16 bytes per lane, non-temporal, one workgroup per CU)"}


def learned_form(w, target, x, q, args, name, force_mode):
    """The same workload in the same precision at the parameter network's
    setting for `target` (enuf_select_params with the trained network),
    timed like the main line: the learned-parameter form beside the
    grid-searched one."""
    import copy

    import torch

    from paper_2004_12484_amd import enuf
    from paper_2004_12484_amd import params as P

    fq = float(np.count_nonzero(w.q)) / w.N
    s, method = P.select_params(w.N, w.box, fq, target, model_path=P.MODEL_BIN)
    wl = copy.copy(w)
    wl.alpha, wl.r_c, wl.M, wl.p = s["alpha"], s["r_c"], tuple(s["M"]), s["p"]
    eng = enuf.Enuf(wl.box, wl.N, wl.alpha, wl.r_c, wl.M, wl.p, precision=w.precision, device=x.device,
                    force_mode=force_mode)
    for _ in range(args.warmup):
        E, F, _ = eng.energy_forces(x, q)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        E, F, _ = eng.energy_forces(x, q)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    acc = golden_check(wl, F.double().cpu().numpy(), float(E[0].item()), name=name)
    eng.close()
    return {"ms_per_step": ms, "value": 1000.0 / ms, "unit": "evals/s", "dtype": w.precision, "target": target,
            "selection": method, "setting": {"alpha": s["alpha"], "r_c": s["r_c"], "M": list(s["M"]), "p": s["p"],
                                             "force_mode": force_mode},
            "accuracy": acc}


def fp64_form(w, setting, x32, q32, args, name):
    """The plain FP64 form of the same workload at its own fastest setting
    meeting the same force-error bar (from `bench.py --search --precision
    f64`), timed like the main line over the same number of steps: the
    comparison the FP32 form has to win at equal stated accuracy."""
    import copy

    import torch

    from paper_2004_12484_amd import enuf

    w64 = copy.copy(w)
    w64.alpha, w64.r_c, w64.M, w64.p = setting["alpha"], setting["r_c"], tuple(setting["M"]), setting["p"]
    x = torch.tensor(w.x, dtype=torch.float64, device=x32.device)
    q = torch.tensor(w.q, dtype=torch.float64, device=x32.device)
    eng = enuf.Enuf(w64.box, w64.N, w64.alpha, w64.r_c, w64.M, w64.p, precision="f64", device=x32.device,
                    force_mode=setting["force_mode"])
    for _ in range(args.warmup):
        E, F, _ = eng.energy_forces(x, q)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        E, F, _ = eng.energy_forces(x, q)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    acc = golden_check(w64, F.cpu().numpy(), float(E[0].item()), name=name)
    eng.close()
    return {"ms_per_step": ms, "value": 1000.0 / ms, "unit": "evals/s", "dtype": "f64",
            "setting": dict(setting), "accuracy": acc}


SEARCH_GRID = dict(mode=("ik", "analytic"), M=(128, 256), p=(4, 6), r_c=(1.5, 1.8, 2.1, 2.4, 2.7, 3.0),
                   alpha_rc=(2.6, 2.9, 3.2))


def search(args, target=1e-4, steps=5):
    """Grid search over ENUF settings for one workload (FP32 unless
    --precision says otherwise): each setting is timed over `steps`
    evaluations (HIP events around the calls) and its RMS force error taken
    against the stored oracle forces."""
    import itertools

    import torch

    from paper_2004_12484_amd import enuf, inputs

    spec = WORKLOADS[args.workload]
    w0 = getattr(inputs, spec["gen"])(**spec["kw"])
    dev = torch.device("cuda", 0)
    prec = args.precision or "f32"
    dt = torch.float64 if prec == "f64" else torch.float32
    x = torch.tensor(w0.x, dtype=dt, device=dev)
    q = torch.tensor(w0.q, dtype=dt, device=dev)
    best = None
    for mode, M, p, rc, arc in itertools.product(*SEARCH_GRID.values()):
        if rc > 0.5 * float(np.min(w0.box)):
            continue
        alpha = arc / rc
        eng = enuf.Enuf(w0.box, w0.N, alpha, rc, (M, M, M), p, precision=prec, device=dev, force_mode=mode)
        for _ in range(2):
            E, F, _ = eng.energy_forces(x, q)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(steps):
            E, F, _ = eng.energy_forces(x, q)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        eng.close()
        w0.alpha, w0.r_c, w0.M, w0.p = alpha, rc, (M, M, M), p
        acc = golden_check(w0, F.double().cpu().numpy(), float(E[0].item()))
        err = acc["rms_force_err"] if acc else None
        rec = {"precision": prec, "force_mode": mode, "M": M, "p": p, "r_c": rc, "alpha": alpha, "ms": ms,
               "rms_force_err": err, "energy_rel_err": acc.get("energy_rel_err") if acc else None}
        print(json.dumps(rec), flush=True)
        if err is not None and err <= target and (best is None or ms < best["ms"]):
            best = rec
    print(json.dumps({"search_best": best, "target": target, "workload": args.workload, "precision": prec}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ions_1m", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=[None, "f32", "f64"])
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--r-c", type=float, default=None)
    ap.add_argument("--M", type=int, default=None)
    ap.add_argument("--p", type=int, default=None)
    ap.add_argument("--force-mode", default=None, choices=["ik", "analytic"],
                    help="reciprocal forces: ik fields (three inverse transforms) or the analytic window "
                         "derivative (one); default: the workload's")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true",
                    help="skip timing the plain FP64 form of the workload beside the main line")
    ap.add_argument("--search", action="store_true",
                    help="grid-search (alpha, r_c, M, p) for the workload: time each FP32 setting and its "
                         "RMS force error against the stored oracle forces; print one JSON line per setting")
    ap.add_argument("--copy-probe", type=float, default=None, metavar="MIB",
                    help="only run a plain device copy of this many MiB (5 times): the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path, "
              "and the figure it reports is one GPU's throughput.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_probe is not None:
        n = int(args.copy_probe * 2 ** 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}), flush=True)
        return

    from paper_2004_12484_amd import enuf, inputs

    if args.search:
        search(args)
        return

    spec = WORKLOADS[args.workload]
    kw = dict(spec["kw"])
    for key, val in (("alpha", args.alpha), ("r_c", args.r_c), ("M", args.M), ("p", args.p)):
        if val is not None:
            kw[key] = val
    if args.precision is not None:
        kw["precision"] = args.precision
    w = getattr(inputs, spec["gen"])(**kw)
    selection = None
    if spec.get("select") and args.alpha is None:
        from paper_2004_12484_amd import params as P

        pred = P.Predictor() if os.path.exists(P.MODEL_PATH) else None
        s, selection = P.choose(w.x, w.q, w.box, spec["select"], predictor=pred)
        w.alpha, w.r_c, w.M, w.p = s["alpha"], s["r_c"], tuple(s["M"]), s["p"]
        selection["target"] = spec["select"]
    dt = torch.float64 if w.precision == "f64" else torch.float32
    rs = 8 if w.precision == "f64" else 4
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    x = torch.tensor(w.x, dtype=dt, device=dev)
    q = torch.tensor(w.q, dtype=dt, device=dev)
    force_mode = args.force_mode or spec.get("force_mode", "ik")
    eng = enuf.Enuf(w.box, w.N, w.alpha, w.r_c, w.M, w.p, precision=w.precision, device=dev,
                    force_mode=force_mode, slater=spec.get("slater"))
    E = torch.empty(5, dtype=torch.float64, device=dev)
    F = torch.empty((w.N, 3), dtype=dt, device=dev)
    phi = torch.empty(w.N, dtype=dt, device=dev) if spec.get("potential") else None
    lib = enuf.load_library()

    def step():
        st = lib.enuf_energy_forces(eng._h, enuf._ptr(x), enuf._ptr(q), enuf._ptr(E), enuf._ptr(F),
                                    enuf._ptr(phi) if phi is not None else None)
        if st != 0:
            enuf._check(st, eng._h)

    eng._bind_stream()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if eng.flags() != 0:
        raise RuntimeError("non-finite input flagged")
    # timed region: K evaluations bracketed by device synchronisation, with
    # nothing else on the stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    # per-phase times: the same K evaluations again with the library's HIP
    # events between phases (on its own streams).  Each event is a marker the
    # command processor waits on, ~5 us apiece, so they stay out of the
    # timed region above.
    eng.set_option(enuf.OPT_TIMING, args.steps)
    torch.cuda.synchronize()
    ep0 = torch.cuda.Event(enable_timing=True)
    ep1 = torch.cuda.Event(enable_timing=True)
    ep0.record()
    for _ in range(args.steps):
        step()
    ep1.record()
    torch.cuda.synchronize()
    ms_phased = ep0.elapsed_time(ep1) / args.steps
    per_step = eng.step_timings(args.steps)          # [K, phases] ms, HIP events on the library's stream
    eng.set_option(enuf.OPT_TIMING, 0)
    phases = {k: float(v) for k, v in zip(enuf.PHASES, per_step.mean(axis=0))}
    step_ms = per_step.sum(axis=1)
    ms = ms_total / args.steps
    value = 1000.0 / ms

    copy = copy_probe(dev)
    counts = eng.stage(enuf.STAGE_COUNTS).cpu().numpy()
    nq = int(counts[1])
    Eh = E.cpu().numpy()
    Fh = F.double().cpu().numpy()
    acc = golden_check(w, Fh, float(Eh[0]), phi.double().cpu().numpy() if phi is not None else None,
                       name=spec.get("golden", args.workload))

    # roofline of the dominant phase
    analytic = force_mode == "analytic"
    ab = algorithmic_bytes(w, rs, nq, nfield=1 if analytic else (4 if phi is not None else 3),
                           out_reals=1 if analytic else 4)
    dom = max(phases, key=phases.get)
    if dom in ab:
        achieved = ab[dom] / (phases[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload, dom),
                "bytes_per_launch": ab[dom], "frac_of_copy": achieved / copy["gbs"]}
    else:
        pairs = pair_count(w, nq)
        peak = FP32_VALU_TFLOPS if rs == 4 else FP64_VALU_TFLOPS
        achieved = pairs * PAIR_FLOPS / (phases[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": measured_traffic(args.workload, dom),
                "flops_per_launch": pairs * PAIR_FLOPS, "unordered_pairs": pairs}
    hbm = {k: ab[k] / (phases[k] * 1e-3) / 1e9 for k in ab}
    # the HBM-bound gates: spread and gather against the HBM peak, with the
    # counter bytes of their kernels beside them when measured on this build
    gates = {k: {"algorithmic_bytes": ab[k], "ms": phases[k], "gbs": hbm[k], "frac": hbm[k] / HBM_PEAK_GBS,
                 "frac_of_copy": hbm[k] / copy["gbs"], "counter_bytes": measured_traffic(args.workload, k)}
             for k in ("spread", "gather")}

    rec = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if rs == 4 else "f64", "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "n_charged": nq, "box": [float(b) for b in w.box],
                   "M": list(w.M), "p": w.p, "alpha": w.alpha, "r_c": w.r_c, "precision": w.precision,
                   "force_mode": force_mode, "potentials": phi is not None, "selection": selection,
                   "slater": spec.get("slater"),
                   "seed": w.seed, "parallelism": "single GPU"},
        "ns_per_particle": ms * 1e6 / w.N, "ns_per_charged": ms * 1e6 / max(nq, 1),
        "wall_s": wall, "step_ms": {"median": float(np.median(step_ms)), "p10": float(np.percentile(step_ms, 10)),
                                    "p90": float(np.percentile(step_ms, 90)), "mean": float(step_ms.mean()),
                                    "with_phase_events": ms_phased},
        "phase_ms": phases, "phase_gbs": hbm, "hbm_gates": gates, "copy_probe": copy,
        "energy": {"total": float(Eh[0]), "real": float(Eh[1]), "recip": float(Eh[2]), "self": float(Eh[3]),
                   "background": float(Eh[4])},
        "accuracy": acc, "roofline": roof,
    }
    if spec.get("learned_form") and not args.no_fp64_form:
        # the network's labels come from ik-force sweeps: its setting is run
        # in that mode
        rec["learned_form"] = learned_form(w, spec["learned_form"], x, q, args, spec.get("golden", args.workload),
                                           "ik")
    if spec.get("fp64_form") and not args.no_fp64_form and w.precision == "f32":
        rec["fp64_form"] = fp64_form(w, spec["fp64_form"], x, q, args, name=spec.get("golden", args.workload))
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
