"""Training and evaluation of the learned block-Jacobi correction.

The network (include/ba.h, BA_PRECOND_LEARNED) is trained on reduced camera
systems the solver itself forms: every scene of the preconditioner stream
(synthetic workload 4: laps of ~200 cameras with loop closures, log-uniform
sizes) takes LM steps 1-5 from its initial estimate with plain block-Jacobi
(mixed precision), and the network inputs of each step's damped reduced
system are kept as a training graph.  Training minimises the mean of the
per-system losses with Adam; forward, backward, the averaging of the
gradients and the optimiser step are the library's kernels
(ba_gnn_loss_grad, ba_gnn_adam).  Evaluation revisits the same five systems
of each held-out scene and solves each to a relative residual of 1e-6 with
FP64 block-Jacobi, mixed-precision block-Jacobi and mixed precision with
the learned blocks, reporting PCG iterations and wall-clock (HIP events;
network inference included for the learned form).

    python -m paper_2409_12190_amd.precond_train --train 400 --test 100 \
        --out paper_2409_12190_amd/data/gnn_params.f32
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ba as B


def stream_problem(seed: int, precision=B.BA_MIXED, n_cams=None, n_pts=None, cg_maxiter=1000,
                   precond=B.BA_PRECOND_LEARNED):
    """(scene, problem) of stream scene `seed` with the learned-preconditioner
    buffers; no step taken yet."""
    from synth.scenes import make_scene
    s = make_scene(4, seed=seed, n_cams=n_cams, n_pts=n_pts)
    p = B.Problem.from_scene(s, precision=precision, cg_maxiter=cg_maxiter, precond=precond)
    return s, p


def training_graph(problem: B.Problem) -> B.Graph:
    """One LM step with plain block-Jacobi, then the graph of its system."""
    problem.set_gnn_params(None)
    problem.lm_step()
    return B.Graph(problem)


def training_graphs(problem: B.Problem, steps: int = 5):
    """The graphs of LM steps 1..steps taken with plain block-Jacobi."""
    return [training_graph(problem) for _ in range(steps)]


def init_params(seed: int = 0):
    """He-scaled hidden layers, zero output layer (block-Jacobi at start);
    float32 on the current device."""
    import torch
    g = torch.Generator().manual_seed(seed)
    F, H, O, L = B.BA_GNN_FEATURES, B.BA_GNN_HIDDEN, B.BA_GNN_OUTPUTS, B.BA_GNN_LAYERS
    parts = [torch.randn(H, F, generator=g) * (2.0 / F) ** 0.5, torch.zeros(H)]
    for _ in range(L):
        parts += [torch.randn(H, H, generator=g) * (2.0 / H) ** 0.5,
                  torch.randn(H, H, generator=g) * (2.0 / H) ** 0.5, torch.zeros(H)]
    parts += [torch.zeros(O, H), torch.zeros(O)]
    theta = torch.cat([t.reshape(-1) for t in parts]).to(torch.float32)
    assert theta.numel() == B.gnn_num_params()
    return theta.cuda()


def mean_loss(graphs, params) -> float:
    import torch
    g = torch.zeros_like(params)
    return float(np.mean([gr.loss_grad(params, g) for gr in graphs]))


def train(graphs, params, epochs: int = 60, lr: float = 2e-3, log=None):
    """Full-batch Adam on the mean loss over the graphs; returns the loss
    history (one value per epoch, before the update).  The gradients of the
    graphs are summed by ba_gnn_loss_grad; ba_gnn_adam takes the mean by its
    grad_scale argument."""
    import torch
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    hist = []
    for ep in range(1, epochs + 1):
        grad.zero_()
        tot = 0.0
        for gr in graphs:
            tot += gr.loss_grad(params, grad)
        hist.append(tot / len(graphs))
        B.gnn_adam(params, grad, m, v, ep, lr, grad_scale=1.0 / len(graphs))
        if log and (ep == 1 or ep % 10 == 0 or ep == epochs):
            log(f"[train] epoch {ep} mean loss {hist[-1]:.6f}")
    torch.cuda.synchronize()
    return hist


def timed_solve(problem: B.Problem, blob: bytes, rtol: float, maxiter: int, params=None):
    """From state `blob`, one LM step whose PCG runs to `rtol`: (cg iterations,
    PCG + network milliseconds by HIP events, precond_used).  The best of two
    runs (the first warms caches)."""
    best = None
    for _ in range(2):
        problem.set_state(blob)
        problem.set_cg(rtol, maxiter)
        if problem.opt.precond == B.BA_PRECOND_LEARNED:
            problem.set_gnn_params(params)
        problem.set_profiling(True, phases=["pcg", "precond_net"])
        info = problem.lm_step()
        ph = problem.phase_times()
        problem.set_profiling(False)
        ms = ph["pcg"][0] + ph["precond_net"][0]
        if best is None or ms < best[1]:
            best = (info["cg_iters"], ms, info["precond_used"], info["cg_rel_resid"])
    return best


def evaluate_scene(seed: int, params, steps: int = 5, rtol: float = 1e-6, maxiter: int = 3000,
                   n_cams=None, n_pts=None):
    """Rows (step, cg and ms of FP64 block-Jacobi, mixed block-Jacobi, learned)
    for LM steps 1..steps of held-out scene `seed`: the trajectory is the
    mixed block-Jacobi solver's at the default tolerance; each step's system
    is solved to `rtol` by the three forms from the same state."""
    s, mixed = stream_problem(seed, B.BA_MIXED, n_cams, n_pts, maxiter)
    f64 = B.Problem.from_scene(s, precision=B.BA_FP64, cg_maxiter=maxiter)
    rows = []
    default_rtol = mixed.opt.cg_rtol
    for k in range(steps):
        blob = mixed.get_state()
        it64, ms64, _, _ = timed_solve(f64, blob, rtol, maxiter)
        itbj, msbj, _, _ = timed_solve(mixed, blob, rtol, maxiter, None)
        itl, msl, used, res = timed_solve(mixed, blob, rtol, maxiter, params)
        rows.append(dict(scene=seed, step=k + 1, n_cams=s.n_cams, n_obs=s.n_obs, cg_fp64=it64,
                         ms_fp64=ms64, cg_bj=itbj, ms_bj=msbj, cg_learned=itl, ms_learned=msl,
                         used=used, resid_learned=res))
        # advance along the block-Jacobi trajectory
        mixed.set_state(blob)
        mixed.set_cg(default_rtol, maxiter)
        mixed.set_gnn_params(None)
        mixed.lm_step()
    mixed.close()
    f64.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=400)
    ap.add_argument("--test", type=int, default=100)
    ap.add_argument("--steps", type=int, default=5, help="LM steps (systems) per scene")
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=None, help="write the trained parameters (raw float32)")
    ap.add_argument("--params", default=None, help="evaluate these parameters (raw float32), no training")
    args = ap.parse_args(argv)
    import torch

    def log(m):
        print(m, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    if args.params:
        params = torch.from_numpy(np.fromfile(args.params, dtype=np.float32)).cuda()
        hist = [float("nan")]
    else:
        graphs = []
        for k in range(args.train):
            s, p = stream_problem(k)
            graphs += training_graphs(p, args.steps)
            p.close()
            if (k + 1) % 50 == 0:
                log(f"[systems] {k + 1}/{args.train} scenes, {len(graphs)} systems "
                    f"({time.perf_counter() - t0:.0f} s)")
        params = init_params()
        hist = train(graphs, params, args.epochs, args.lr, log)
        for g in graphs:
            g.close()
        del graphs
        if args.out:
            params.cpu().numpy().astype(np.float32).tofile(args.out)
    rows = []
    for k in range(args.train, args.train + args.test):
        rows += evaluate_scene(k, params, args.steps)
        if (k + 1 - args.train) % 25 == 0:
            log(f"[eval] {k + 1 - args.train}/{args.test} ({time.perf_counter() - t0:.0f} s)")
    col = lambda key: np.array([r[key] for r in rows], dtype=np.float64)  # noqa: E731
    out = {
        "train_scenes": args.train, "test_scenes": args.test, "systems_per_scene": args.steps,
        "epochs": args.epochs, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
        "test_systems": len(rows),
        "cg_iters_mean": {"fp64_block_jacobi": col("cg_fp64").mean(), "mixed_block_jacobi": col("cg_bj").mean(),
                          "mixed_learned": col("cg_learned").mean()},
        "ms_mean": {"fp64_block_jacobi": col("ms_fp64").mean(), "mixed_block_jacobi": col("ms_bj").mean(),
                    "mixed_learned": col("ms_learned").mean()},
        "ms_total": {"fp64_block_jacobi": col("ms_fp64").sum(), "mixed_block_jacobi": col("ms_bj").sum(),
                     "mixed_learned": col("ms_learned").sum()},
        "systems_learned_faster_than_mixed_bj": int((col("ms_learned") < col("ms_bj")).sum()),
        "fallbacks_to_block_jacobi": int((col("used") == 2).sum()),
        "max_resid_learned": float(col("resid_learned").max()),
        "wall_s": time.perf_counter() - t0,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
