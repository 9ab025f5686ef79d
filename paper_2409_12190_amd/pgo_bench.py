"""Timing of the pose-graph LM iteration (ba_pgo_*) on synthetic sphere graphs.

Each graph (rings x per_ring poses on a sphere, odometry plus loop closures
to the previous ring; the default 50 x 50 has the size of the paper's sphere
benchmark, 2,500 poses / 9,800 edges) is solved from its dead-reckoning
start with the library's LM iteration (FP64 and mixed storage, pipelined
PCG, rtol 1e-4, 250 iterations at most), after one untimed pass over the
same steps; the time per LM step comes from HIP events on the problem's
stream around every phase (and the wall clock around the steps).  Prints
one JSON line.

    python -m paper_2409_12190_amd.pgo_bench [--rings 50 --per-ring 50 --steps 10]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rings", type=int, default=50)
    ap.add_argument("--per-ring", type=int, default=50)
    ap.add_argument("--steps", type=int, default=10)
    args = ap.parse_args()

    import torch

    from paper_2409_12190_amd import ba as B
    from synth.posegraph import make_pose_graph

    g = make_pose_graph(0, rings=args.rings, per_ring=args.per_ring)
    out = {"graph": {"poses": g.n_poses, "edges": g.n_edges, "rings": args.rings,
                     "per_ring": args.per_ring}, "steps": args.steps, "forms": {}}
    for name, prec in (("fp64", B.BA_FP64), ("mixed", B.BA_MIXED)):
        with B.PoseGraph.from_graph(g, precision=prec) as p:
            for _ in range(args.steps):  # untimed pass (code objects, caches)
                p.lm_step()
            p.set_poses(g.poses0)
            p.set_lambda(1e-4)
            p.set_profiling(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = [p.lm_step() for _ in range(args.steps)]
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ph = {k: v for k, v in p.phase_times().items() if v[1] > 0}
            gpu_ms = sum(v[0] for v in ph.values()) / args.steps
            last = infos[-1]
            out["forms"][name] = {
                "ms_per_step_events": round(gpu_ms, 4), "ms_per_step_wall": round(wall / args.steps * 1e3, 4),
                "cg_iters_per_step": sum(i["cg_iters"] for i in infos) / args.steps,
                "cost_after": last["cost_after"] if last["accepted"] else last["cost_before"],
                "plan": p.plan,
                "phases_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in ph.items()}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
