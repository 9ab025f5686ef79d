#!/usr/bin/env python3
"""Throughput of the bundle-adjustment LM iteration on one MI355X.

A step is one Levenberg-Marquardt iteration (ba_lm_step) over the whole
synthetic scene: residuals and Jacobian blocks, J^T J / J^T r assembly, Schur
complement onto the cameras, block-Jacobi PCG, back-substitution, candidate
cost and acceptance.  Inputs are resident in HBM before the timed region.

Default workload: the largest single scene, 10,000 cameras in 10 laps of a
circuit, 2,000,000 points (about 8.0M observations, banded co-visibility plus
5% loop-closure observations), Huber loss (1 px), mixed precision (FP32
Jacobian / Schur storage, FP64 arithmetic and reductions), compared with
plain FP64 and, when trained parameters are present, with the learned
preconditioner, on the same GPU.  Value = observations x LM iterations /
second of the mixed form.  Prints one JSON line.
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
    if name == "linearize":   # obs xy, w, indices in; w, observation row (Jc, Jp, Q, w) and
        # record (r, w, e) out; cameras and points in; V, gp, Vinv, ep per point out
        return (no * (16 + 8 + 4 + 4 + 8 + 31 * es + 40) + nc * 80
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
    # (the plan decides which blocks and columns each PCG workgroup moves)
    "pcg": ("ba_pcg.hip", "ba_reduce.h", "ba_kernels.h", "ba_internal.h", "ba_plan.cpp"),
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


def recorded_traffic(workload, kernel, cg_iters=None):
    """Per-launch HBM bytes of a kernel from the counter summary under
    profiles/ (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading),
    or None when the summary is absent or was taken on other sources.  A
    summary that gives bytes per CG iteration is scaled to the launch's
    cg_iters."""
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
        if cg_iters is not None and "bytes_per_cg_iteration" in vals:
            return float(vals["bytes_per_cg_iteration"]) * cg_iters
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


def cost_after(info):
    return info["cost_after"] if info["accepted"] else info["cost_before"]


def first_reaching(infos, times, target):
    t = 0.0
    for i, (inf, dt) in enumerate(zip(infos, times)):
        t += dt
        if cost_after(inf) <= target:
            return i + 1, t
    return None, None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    """Cores this process may use: the affinity mask, capped by
    OMP_NUM_THREADS when the environment sets the host's share."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(scene, iters, single_iters, it_bytes_fn, repeats=1):
    """The FP64 oracle on the host's cores: `iters` LM iterations of the
    whole scene at all cores (also the FP64 reference cost after them), then
    `single_iters` at one thread (bounded sample); each timed `repeats`
    times from the initial state, the median kept (the oracle's results do
    not depend on the thread count or the repeat)."""
    from oracle import oracle as O
    nproc = host_cores()
    out = {}
    for threads, n in ((nproc, iters), (1, single_iters)):
        if n <= 0:
            continue
        O.set_threads(threads)
        times = []
        for _ in range(max(1, repeats)):
            o = O.Oracle.from_scene(scene, options=O.OracleOptions(huber_delta=scene.huber_delta))
            t0 = time.perf_counter()
            infos = []
            for _ in range(n):
                infos.append(o.lm_step())
            times.append(time.perf_counter() - t0)
            del o
        el = sorted(times)[len(times) // 2]
        cg = sum(i["cg_iters"] for i in infos) / n
        out[threads] = dict(s=el, runs=[round(t, 2) for t in times], iters=n, cost=cost_after(infos[-1]),
                            cg=cg, gbs=it_bytes_fn(cg) * n / el / 1e9)
        log(f"[bench] oracle at {threads} threads: {n} LM iterations, median {el:.2f} s of {[round(t, 2) for t in times]} "
            f"(cost {out[threads]['cost']:.9e})")
    O.set_threads(nproc)
    return out


def learned_params_path():
    return os.path.join(ROOT, "paper_2409_12190_amd", "data", "gnn_params.f32")


def load_learned_params():
    """Trained network parameters (raw float32, written by precond_train
    --out), or None."""
    import numpy as np
    import torch
    from paper_2409_12190_amd import ba as B
    path = learned_params_path()
    if not os.path.exists(path):
        return None
    v = np.fromfile(path, dtype=np.float32)
    if v.size != B.gnn_num_params():
        return None
    return torch.from_numpy(v).cuda()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="laps10000")
    ap.add_argument("--cpu-iters", type=int, default=-1,
                    help="LM iterations of the oracle at all host cores (-1: the workload's "
                         "reference iterations; 0 disables the CPU legs)")
    ap.add_argument("--cpu-single-iters", type=int, default=1,
                    help="LM iterations of the oracle at one thread (bounded sample)")
    ap.add_argument("--cpu-repeats", type=int, default=3,
                    help="timed runs of each CPU leg (the median is reported)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
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
    K = args.steps

    learned = None if args.skip_learned else load_learned_params()
    forms_todo = [("fp64", B.BA_FP64, False), ("mixed", B.BA_MIXED, False)]
    if args.skip_fp64:
        forms_todo = forms_todo[1:]
    if learned is not None:
        forms_todo.append(("learned", B.BA_MIXED, True))
    forms = {}
    for name, prec, use_net in forms_todo:
        t = time.perf_counter()
        kw = dict(precond=B.BA_PRECOND_LEARNED) if use_net else {}
        prob = B.Problem.from_scene(scene, precision=prec, **kw)
        if use_net:
            prob.set_gnn_params(learned)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t
        log(f"[bench] {name}: setup {setup:.2f} s (symbolic analysis + upload), nnzb={prob.nnzb}, "
            f"plan {prob.plan}")
        if args.warmup:
            run_steps(prob, args.warmup, scene.cams0, scene.pts0, 1e-4)
        # timed run of K steps: events only around the PCG (the dominant
        # kernel's live duration); the run then continues untimed by events
        # until twice the reference iterations, so that the time to the FP64
        # reference cost is measured when a form needs more iterations; then
        # the same K steps again with every phase bracketed (breakdown)
        steps = max(K, ref_iters) if name == "fp64" else max(K, 2 * ref_iters)
        prob.set_profiling(True, phases=["pcg"])
        infos, times, total = run_steps(prob, K, scene.cams0, scene.pts0, 1e-4)
        timed_phases = prob.phase_times()
        prob.set_profiling(False)
        if steps > K:
            more_infos, more_times = continue_steps(prob, steps - K)
            infos += more_infos
            times += more_times
        prob.set_profiling(True)
        run_steps(prob, K, scene.cams0, scene.pts0, 1e-4)
        phases = prob.phase_times()
        phases["pcg"] = timed_phases["pcg"]
        prob.set_profiling(False)
        k_time = sum(times[:K])
        log(f"[bench] {name}: {steps} steps, first {K} in {k_time*1e3:.1f} ms, "
            f"cost after {ref_iters}: {cost_after(infos[ref_iters - 1]):.9e}")
        forms[name] = dict(prob=prob, infos=infos, times=times, phases=phases, k_time=k_time,
                           setup=setup, plan=prob.plan, nnzb=prob.nnzb)

    mixed = forms["mixed"]
    value = scene.n_obs * K / mixed["k_time"]
    out = {
        "metric": METRIC, "value": value, "unit": "obs*LM-iters/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": mixed["k_time"] / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 arithmetic, f32 storage of J and S",
        "data": "synthetic (seeded generator, structure of the workload; no dataset)",
        "config": {"workload": CONFIG_NAMES[cfg], "n_cams": scene.n_cams, "n_pts": scene.n_pts,
                   "n_obs": scene.n_obs,
                   "precision": "mixed (fp32 J/S storage, fp64 arithmetic, reductions and CG vectors)",
                   "loss": f"huber {scene.huber_delta}" if scene.huber_delta > 0 else "l2",
                   "cg": "block-Jacobi PCG (pipelined recurrence), rtol 1e-4, maxiter 250",
                   "pcg_layout": mixed["plan"]["pcg_layout"]},
    }
    # per-phase breakdown and the dominant kernel's roofline
    es = 4
    nnzb = mixed["nnzb"]
    cg_total = sum(i["cg_iters"] for i in mixed["infos"][:K])
    ph = {k: v for k, v in mixed["phases"].items() if v[1] > 0}
    out["phases_ms_per_step"] = {k: round(v[0] / K, 4) for k, v in ph.items()}
    dom = max(ph, key=lambda k: ph[k][0])
    ms, n = ph[dom]
    t = np.bincount(scene.pt_idx, minlength=scene.n_pts).astype(np.int64)
    n_pairs = int((t * (t + 1) // 2).sum())   # (x, y) pairs with camera(x) <= camera(y)
    per_launch = kernel_bytes(dom, scene, nnzb, n_pairs, es, cg_total / max(n, 1))
    if per_launch is not None:
        achieved = per_launch / (ms / n * 1e-3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS,
                           "traffic": recorded_traffic(args.workload, dom, cg_total / max(n, 1)),
                           "kernel": dom, "avg_launch_ms": ms / n, "launches": n,
                           "algorithmic_bytes_per_launch": per_launch,
                           "cg_iters_per_launch": cg_total / max(n, 1)}
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
    out["forms"] = {}
    for name, f in forms.items():
        out["forms"][name] = {
            "value": scene.n_obs * K / f["k_time"], "ms_per_step": f["k_time"] / K * 1e3,
            "cg_iters_per_step": sum(i["cg_iters"] for i in f["infos"][:K]) / K,
            "pcg_layout": f["plan"]["pcg_layout"],
            "cost_after_ref_iters": cost_after(f["infos"][ref_iters - 1]),
            "phases_ms_per_step": {k: round(v[0] / K, 4) for k, v in f["phases"].items() if v[1] > 0}}
    if "learned" in forms:
        used = [i["precond_used"] for i in forms["learned"]["infos"]]
        out["forms"]["learned"]["steps_by_preconditioner"] = {
            "learned": used.count(1), "fallback_block_jacobi": used.count(2), "block_jacobi": used.count(0)}
        out["forms"]["learned"]["params"] = os.path.relpath(learned_params_path(), ROOT)
    if "fp64" in forms:
        f64 = forms["fp64"]
        F_ref = min(cost_after(i) for i in f64["infos"][:ref_iters])
        target = F_ref * (1 + 1e-6)
        out["reference_cost_fp64"] = F_ref
        tt = {}
        for name, f in forms.items():
            its, secs = first_reaching(f["infos"], f["times"], target)
            tt[name] = {"s": secs, "iters": its}
        out["time_to_1e-6_rel_cost"] = tt
        t64 = tt["fp64"]["s"]
        out["speedup_vs_fp64"] = {name: (t64 / tt[name]["s"]) if (t64 and tt[name]["s"]) else None
                                  for name in forms if name != "fp64"}
        out["per_step_speedup_vs_fp64"] = f64["k_time"] / mixed["k_time"]
    for f in forms.values():
        f["prob"].close()
    cpu_iters = ref_iters if args.cpu_iters < 0 else args.cpu_iters
    if cpu_iters > 0:
        log("[bench] CPU baseline (oracle)")
        res = cpu_baseline(scene, cpu_iters, args.cpu_single_iters,
                           lambda cg: iteration_bytes(scene, nnzb, 8, cg), args.cpu_repeats)
        nproc = host_cores()
        full = res[nproc]
        out["cpu_baseline"] = {
            "value": scene.n_obs * full["iters"] / full["s"], "unit": "obs*LM-iters/s", "cores": nproc,
            "kind": "oracle",
            "sample": f"{full['iters']} LM iterations of the whole scene from its initial state, FP64 "
                      f"C oracle (OpenMP, results independent of the thread count), median {full['s']:.1f} s "
                      f"of runs {full['runs']}",
            "cpu_model": cpu_model(), "effective_GB/s": round(full["gbs"], 2)}
        if 1 in res and nproc != 1:
            one = res[1]
            out["cpu_baseline"]["single_thread"] = {
                "value": scene.n_obs * one["iters"] / one["s"], "cores": 1,
                "sample": f"{one['iters']} LM iteration(s) from the initial state, median {one['s']:.1f} s "
                          f"of runs {one['runs']}",
                "effective_GB/s": round(one["gbs"], 2)}
        if full["iters"] >= ref_iters:
            F_o = full["cost"]
            out["oracle_cost_after_ref_iters"] = F_o
            out["final_cost_error_vs_oracle"] = {
                name: abs(f["cost_after_ref_iters"] - F_o) / F_o for name, f in out["forms"].items()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
