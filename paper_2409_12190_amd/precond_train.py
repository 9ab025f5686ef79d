"""Training and evaluation of the learned block-Jacobi correction.

The network (include/ba.h, BA_PRECOND_LEARNED) is trained on reduced camera
systems the solver itself forms: for every scene of the preconditioner
stream (synthetic workload 4) one LM step is taken from the initial
estimate, and the network inputs of that step's damped reduced system are
kept as a training graph.  Training minimises the mean of the per-system
losses with Adam; forward, backward and the optimiser step are the
library's kernels (ba_gnn_loss_grad, ba_gnn_adam).  Evaluation solves the
first-step system of held-out scenes to a relative residual of 1e-6 with
block-Jacobi and with the learned blocks and reports PCG iterations and
wall-clock (network included).

    python -m paper_2409_12190_amd.precond_train --train 400 --test 100 --out params.pt
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import ba as B


def stream_problem(seed: int, precision=B.BA_MIXED, n_cams=None, n_pts=None, cg_maxiter=1000):
    """(scene, problem) of stream scene `seed` with the learned-preconditioner
    buffers; no step taken yet."""
    from synth.scenes import make_scene
    s = make_scene(4, seed=seed, n_cams=n_cams, n_pts=n_pts)
    p = B.Problem.from_scene(s, precision=precision, cg_maxiter=cg_maxiter,
                             precond=B.BA_PRECOND_LEARNED)
    return s, p


def training_graph(problem: B.Problem) -> B.Graph:
    """One LM step with plain block-Jacobi, then the graph of its system."""
    problem.set_gnn_params(None)
    problem.lm_step()
    return B.Graph(problem)


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
    history (one value per epoch, before the update)."""
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
        grad /= len(graphs)
        hist.append(tot / len(graphs))
        B.gnn_adam(params, grad, m, v, ep, lr)
        if log and (ep == 1 or ep % 10 == 0 or ep == epochs):
            log(f"[train] epoch {ep} mean loss {hist[-1]:.6f}")
    torch.cuda.synchronize()
    return hist


def solve_first_step(scene, problem: B.Problem, params, rtol: float = 1e-6, maxiter: int = 1000):
    """The first LM step's PCG to `rtol` with block-Jacobi (params None) or the
    learned blocks: (cg iterations, PCG + network milliseconds, precond_used)."""
    problem.set_params(scene.cams0, scene.pts0)
    problem.set_lambda(1e-4)
    problem.set_cg(rtol, maxiter)
    problem.set_gnn_params(params)
    problem.set_profiling(True)
    info = problem.lm_step()
    ph = problem.phase_times()
    problem.set_profiling(False)
    ms = ph["pcg"][0] + ph["precond_net"][0]
    return info["cg_iters"], ms, info["precond_used"]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=400)
    ap.add_argument("--test", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None, help="write the trained parameters (torch.save)")
    args = ap.parse_args(argv)
    import torch

    def log(m):
        print(m, file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    graphs = []
    for k in range(args.train):
        s, p = stream_problem(k)
        graphs.append(training_graph(p))
        del p
        if (k + 1) % 50 == 0:
            log(f"[systems] {k + 1}/{args.train} training systems ({time.perf_counter() - t0:.0f} s)")
    params = init_params()
    hist = train(graphs, params, args.epochs, args.lr, log)
    del graphs
    rows = []
    for k in range(args.train, args.train + args.test):
        s, p = stream_problem(k)
        it_bj, ms_bj, _ = solve_first_step(s, p, None)
        it_l, ms_l, used = solve_first_step(s, p, params)
        rows.append((s.n_cams, s.n_pts, s.n_obs, it_bj, it_l, ms_bj, ms_l, used))
        del p
        if (k + 1 - args.train) % 25 == 0:
            log(f"[eval] {k + 1 - args.train}/{args.test}")
    r = np.array(rows, dtype=np.float64)
    out = {
        "train_scenes": args.train, "test_scenes": args.test, "epochs": args.epochs,
        "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
        "cg_iters_block_jacobi_mean": float(r[:, 3].mean()), "cg_iters_learned_mean": float(r[:, 4].mean()),
        "cg_iters_ratio_mean": float((r[:, 4] / r[:, 3]).mean()),
        "ms_block_jacobi_mean": float(r[:, 5].mean()), "ms_learned_mean": float(r[:, 6].mean()),
        "fallbacks": int((r[:, 7] == 2).sum()),
        "wall_s": time.perf_counter() - t0,
    }
    if args.out:
        torch.save(params.cpu(), args.out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
