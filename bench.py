#!/usr/bin/env python3
"""Throughput of the bundle-adjustment LM iteration on one MI355X.

A step is one Levenberg-Marquardt iteration (ba_lm_step) over the whole
synthetic scene: residuals and Jacobian blocks, J^T J / J^T r assembly, Schur
complement onto the cameras, block-Jacobi PCG, back-substitution, candidate
cost and acceptance.  Inputs are resident in HBM before the timed region.

Default workload: 1,000 cameras on a random-walk trajectory, 200,000 points
with power-law tracks (about 1.0M observations), Huber loss (1 px), mixed
precision (FP32 Jacobian / Schur storage, FP64 arithmetic and reductions),
compared with plain FP64 on the same GPU.  Value = observations x LM
iterations / second of the mixed form.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "obs·LM-iters/sec at 1e-6 rel. cost; mixed/learned vs FP64 block-Jacobi speedup"
WORKLOADS = {"traj1000": 1, "laps10000": 2, "ring16": 0}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(name, scene, nnzb, es, cg_iters):
    """Algorithmic HBM bytes of one launch of a phase (each input read once,
    each output written once; see the design notes for the derivation)."""
    no, nc, np_ = scene.n_obs, scene.n_cams, scene.n_pts
    nnz_off = nnzb - nc
    if name == "linearize":
        return no * (16 + 8 + 4 + 4 + 16 + 8 + 24 * es) + nc * 80 + np_ * (24 + 72)
    if name == "camera_diag":
        return no * (4 + 4 + 24 * es + 8 + 16) + np_ * (48 + 24) + nc * (81 * es + 3 * 72 + 648)
    if name == "schur_offdiag":
        return no * (4 + 24 * es + 8) + np_ * 48 + nnz_off * 81 * es
    if name == "pcg":
        s_bytes = (nnz_off * 81 + nc * 45) * es
        per_iter = s_bytes + nc * 45 * 8 + 8 * nc * 9 * 8
        return cg_iters * per_iter + nc * 9 * 8 * 5
    if name == "backsub":
        return no * (4 + 4 + 24 * es + 8) + nc * 72 + np_ * (24 + 48 + 24 + 24 + 24)
    if name == "candidate_cost":
        return no * (16 + 8 + 4 + 4) + nc * 80 + np_ * 24
    return None


def run_steps(prob, steps, cams0, pts0, lam0):
    import torch
    prob.set_params(cams0, pts0)
    prob.set_lambda(lam0)
    torch.cuda.synchronize()
    infos, times = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        infos.append(prob.lm_step())
        times.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    return infos, times, time.perf_counter() - t0


def first_reaching(infos, times, target):
    t = 0.0
    for i, (inf, dt) in enumerate(zip(infos, times)):
        t += dt
        F = inf["cost_after"] if inf["accepted"] else inf["cost_before"]
        if F <= target:
            return i + 1, t
    return None, None


def cpu_baseline(scene, budget_s):
    from oracle import oracle as O
    o = O.Oracle.from_scene(scene, options=O.OracleOptions(huber_delta=scene.huber_delta))
    t0 = time.perf_counter()
    n = 0
    while True:
        o.lm_step()
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= scene.lm_iters:
            break
    return {"value": scene.n_obs * n / el, "unit": "obs*LM-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} LM iterations of the full scene from its initial state "
                      f"({el:.1f} s, single-threaded FP64 C oracle)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="traj1000")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 disables it)")
    ap.add_argument("--skip-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            f"(asked for --gpus {args.gpus}).")
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_12190_amd import ba as B
    from synth.scenes import CONFIG_NAMES, make_scene

    torch.cuda.set_device(0)
    cfg = WORKLOADS[args.workload]
    log(f"[bench] generating workload {CONFIG_NAMES[cfg]}")
    scene = make_scene(cfg)
    log(f"[bench] n_cams={scene.n_cams} n_pts={scene.n_pts} n_obs={scene.n_obs}")
    ref_iters = scene.lm_iters

    forms = {}
    for name, prec in (("fp64", B.BA_FP64), ("mixed", B.BA_MIXED)):
        if name == "fp64" and args.skip_fp64:
            continue
        t = time.perf_counter()
        prob = B.Problem.from_scene(scene, precision=prec)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t
        log(f"[bench] {name}: setup {setup:.2f} s (symbolic analysis + upload), nnzb={prob.nnzb}")
        if args.warmup:
            run_steps(prob, args.warmup, scene.cams0, scene.pts0, 1e-4)
        prob.set_profiling(True)
        steps = max(args.steps, ref_iters) if name == "fp64" else args.steps
        infos, times, total = run_steps(prob, steps, scene.cams0, scene.pts0, 1e-4)
        phases = prob.phase_times()
        prob.set_profiling(False)
        k_time = sum(times[:args.steps])
        log(f"[bench] {name}: {steps} steps, first {args.steps} in {k_time*1e3:.1f} ms, "
            f"final cost {infos[-1]['cost_after']:.6f}")
        forms[name] = dict(prob=prob, infos=infos, times=times, phases=phases, k_time=k_time,
                           setup=setup)

    mixed = forms["mixed"]
    K = args.steps
    value = scene.n_obs * K / mixed["k_time"]
    out = {
        "metric": METRIC, "value": value, "unit": "obs*LM-iters/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": mixed["k_time"] / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": CONFIG_NAMES[cfg], "n_cams": scene.n_cams, "n_pts": scene.n_pts,
                   "n_obs": scene.n_obs, "precision": "mixed (fp32 J/S storage, fp64 arithmetic)",
                   "loss": f"huber {scene.huber_delta}" if scene.huber_delta > 0 else "l2",
                   "cg": "block-Jacobi PCG, rtol 1e-4, maxiter 250"},
    }
    # per-phase breakdown and the dominant kernel's roofline
    es = 4
    nnzb = mixed["prob"].nnzb
    cg_total = sum(i["cg_iters"] for i in mixed["infos"][:K])
    ph = {k: v for k, v in mixed["phases"].items() if v[1] > 0}
    out["phases_ms_per_step"] = {k: round(v[0] / K, 4) for k, v in ph.items()}
    dom = max(ph, key=lambda k: ph[k][0])
    ms, n = ph[dom]
    per_launch = kernel_bytes(dom, scene, nnzb, es, cg_total / max(n, 1))
    if per_launch is not None:
        achieved = per_launch / (ms / n * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom,
                           "avg_launch_ms": ms / n, "launches": n}
    out["cg_iters_per_step"] = cg_total / K
    out["nnzb"] = nnzb
    out["final_cost_after_K"] = mixed["infos"][K - 1]["cost_after"]
    if "fp64" in forms:
        f64 = forms["fp64"]
        F_ref = min(i["cost_after"] if i["accepted"] else i["cost_before"]
                    for i in f64["infos"][:ref_iters])
        target = F_ref * (1 + 1e-6)
        it64, t64 = first_reaching(f64["infos"], f64["times"], target)
        itm, tm = first_reaching(mixed["infos"], mixed["times"], target)
        out["fp64"] = {"value": scene.n_obs * K / f64["k_time"], "ms_per_step": f64["k_time"] / K * 1e3,
                       "phases_ms_per_step": {k: round(v[0] / len(f64["times"]), 4)
                                              for k, v in f64["phases"].items() if v[1] > 0}}
        out["reference_cost_fp64"] = F_ref
        out["time_to_1e-6_rel_cost_s"] = {"fp64": t64, "mixed": tm, "fp64_iters": it64,
                                          "mixed_iters": itm}
        out["speedup_vs_fp64"] = (t64 / tm) if (t64 and tm) else None
        out["per_step_speedup_vs_fp64"] = f64["k_time"] / mixed["k_time"]
    if args.cpu_budget > 0:
        log("[bench] CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(scene, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
