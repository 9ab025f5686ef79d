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


def kernel_bytes(name, scene, nnzb, n_pairs, es, cg_iters):
    """Algorithmic HBM bytes of one launch of a phase: every input the
    kernel needs read once and every output written once (gathered
    per-point or per-camera data counted once per point or camera).
    es = bytes per stored Jacobian / Q / S value (8 FP64, 4 mixed)."""
    no, nc, np_ = scene.n_obs, scene.n_cams, scene.n_pts
    nnz_off = nnzb - nc
    if name == "linearize":   # obs xy, w, indices in; r, w, observation row (Jc, Jp, Q, w) and
        # record (r, w, e) out; cameras and points in; V, gp, Vinv, ep per point out
        return (no * (16 + 8 + 4 + 4 + 16 + 8 + 31 * es + 40) + nc * 80
                + np_ * (24 + 48 + 24 + 48 + 24))
    if name == "damp_points":  # V, gp in; Vinv, ep out (after a rejected step)
        return np_ * (48 + 24 + 48 + 24)
    if name == "point_q":      # point index, Jp, w in; Q, w, e out; Vinv, ep per point
        return no * (4 + 6 * es + 8 + 7 * es + 16) + np_ * (48 + 24)
    if name == "schur_pairs":  # pair steps; observation rows (Jc, Jp, Q, w) and records
        # (r, w, e) once each; S blocks and the camera vectors (gc, bS, diag U) out
        return (n_pairs * 8 + no * (31 * es + 40)
                + nnz_off * 81 * es + nc * (648 + 216))
    if name == "camera_finish":  # diagonal blocks and diagU in; damped blocks, inverses out
        return nc * (648 + 72 + 648 + 648)
    if name == "pcg":          # per CG iteration: S (upper blocks, symmetric diagonal),
        per_iter = ((nnz_off * 81 + nc * 45) * es   # block-Jacobi factors and the
                    + nc * 45 * es + 8 * nc * 9 * 8)  # FP64 vectors (x, r, z, p, q touches)
        return cg_iters * per_iter + nc * 9 * 8 * 2
    if name == "backsub":      # indices, J, w per observation; dc per camera;
        return no * (4 + 4 + 24 * es + 8) + nc * 72 + np_ * (24 + 48 + 24 + 24 + 24)
    if name == "retract_cameras":
        return nc * (80 + 72 + 80 + 72 + 1)
    if name == "candidate_cost":
        return no * (4 + 4 + 16 + 8) + nc * 80 + np_ * 24
    return None


def iteration_bytes(scene, nnzb, es, cg_iters):
    """Compulsory bytes of one LM iteration (observation stream at the
    current and the candidate parameters, FP64 parameters read twice and
    written once, S written once and read every CG iteration with its
    block-Jacobi factors, FP64 CG vectors); storing J, Q and the per-point
    blocks between kernels is implementation overhead and not counted."""
    no, nc, np_ = scene.n_obs, scene.n_cams, scene.n_pts
    d = 9
    s_x = 8
    b_obs = 2 * no * (8 + 2 * s_x + (s_x if scene.obs_w is not None else 0))
    b_par = 3 * (nc * 80 + np_ * 24)
    b_s = (1 + cg_iters) * ((nnzb - nc) * d * d + nc * d * (d + 1) // 2) * es
    b_pc = cg_iters * nc * d * (d + 1) // 2 * es
    b_vec = cg_iters * 8 * nc * d * 8
    return b_obs + b_par + b_s + b_pc + b_vec


KERNEL_SOURCES = {
    "pcg": ("ba_pcg.hip", "ba_reduce.h", "ba_kernels.h", "ba_internal.h"),
}
DEFAULT_SOURCES = ("ba_kernels.hip", "ba_reduce.h", "ba_kernels.h", "ba_internal.h", "ba_device.h")


def source_digest(kernel="pcg"):
    """Digest of a kernel's sources: HBM traffic counters recorded for other
    sources no longer describe the kernel."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, DEFAULT_SOURCES):
        with open(os.path.join(ROOT, "paper_2409_12190_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, kernel):
    """Per-launch HBM bytes of a kernel from the counter summary under
    profiles/ (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading),
    or None when the summary is absent or was taken on other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_digest") != source_digest(kernel):
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe():
    """A plain device copy of known size (512 MiB read, 512 MiB written),
    the calibration of the HBM byte counters."""
    import torch
    n = 512 << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 5}))


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


def continue_steps(prob, steps):
    """More LM steps from the problem's current state."""
    import torch
    torch.cuda.synchronize()
    infos, times = [], []
    for _ in range(steps):
        a = time.perf_counter()
        infos.append(prob.lm_step())
        times.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    return infos, times


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
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain 512 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            f"(asked for --gpus {args.gpus}).")
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
        return

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
        # timed run of K steps: events only around the PCG (the dominant
        # kernel's live duration); the mixed form then runs on, untimed by
        # events, until twice the reference iterations, so that its time to
        # the FP64 reference cost is measured when it needs more iterations;
        # then the same K steps again with every phase bracketed, for the
        # per-phase breakdown
        if name == "fp64":
            steps = max(args.steps, ref_iters)
        else:
            steps = args.steps if args.skip_fp64 else max(args.steps, 2 * ref_iters)
        prob.set_profiling(True, phases=["pcg"])
        infos, times, total = run_steps(prob, args.steps, scene.cams0, scene.pts0, 1e-4)
        timed_phases = prob.phase_times()
        prob.set_profiling(False)
        if steps > args.steps:
            more_infos, more_times = continue_steps(prob, steps - args.steps)
            infos += more_infos
            times += more_times
        prob.set_profiling(True)
        run_steps(prob, args.steps, scene.cams0, scene.pts0, 1e-4)
        phases = prob.phase_times()
        phases["pcg"] = timed_phases["pcg"]
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
        "data": "synthetic (seeded generator, structure of the workload; no dataset)",
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
    import numpy as np
    t = np.bincount(scene.pt_idx, minlength=scene.n_pts).astype(np.int64)
    n_pairs = int((t * (t + 1) // 2).sum())   # (x, y) pairs with camera(x) <= camera(y)
    per_launch = kernel_bytes(dom, scene, nnzb, n_pairs, es, cg_total / max(n, 1))
    if per_launch is not None:
        achieved = per_launch / (ms / n * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS,
                           "traffic": recorded_traffic(args.workload, dom),
                           "kernel": dom, "avg_launch_ms": ms / n, "launches": n,
                           "algorithmic_bytes_per_launch": per_launch}
    out["phase_roofline"] = {}
    for k, (pms, pn) in ph.items():
        kb = kernel_bytes(k, scene, nnzb, n_pairs, es, cg_total / max(pn, 1))
        if kb is not None:
            gbs = kb / (pms / pn * 1e-3) / 1e9
            out["phase_roofline"][k] = {"GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                                        "avg_launch_us": round(pms / pn * 1e3, 2)}
    it_bytes = iteration_bytes(scene, nnzb, es, cg_total / K)
    it_s = mixed["k_time"] / K
    out["iteration_roofline"] = {"compulsory_bytes": it_bytes, "ms": it_s * 1e3,
                                 "frac": it_bytes / it_s / 1e9 / HBM_PEAK_GBS}
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
                       "phases_ms_per_step": {k: round(v[0] / K, 4)
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
