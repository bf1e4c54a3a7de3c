"""Train the correction network of the learned preconditioner stage on the
device.

Recipe (all seeded):
  1. Flows past the fixed cylinder of the training grid are started
     impulsively at several inflow angles (the body and the grid, and so the
     matrix K, are the same for every run; only the right-hand sides differ).
  2. At a few time steps of each run the right-hand side of the modified
     Poisson system (Eq. 11b) is formed with the library's stages, solved to
     a 1e-12 relative residual (x*), and an AMG-PCG solve from the previous
     lambda is replayed with ibpm_harvest, which stores before each iteration
     the residual left by one V-cycle, r1 = r - K V(r), and the error that
     remains, e1 = x* - x - V(r).  Every k-th pair is kept.
  3. The network is trained on these pairs with Adam (ibpm_nn_train) on the
     energy-norm loss (the share of the error that the optimally scaled
     correction removes), the pairs shuffled by a seeded generator each
     epoch, the learning rate halved at fixed epochs.

The weights are written as a float32 .npy file of IBPM_NN_PARAMS values and
a JSON record of the recipe, pair counts and losses.

    python -m paper_1109_3524_amd.train_learned --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import ibpm
from . import workloads as W


def training_workload(alpha: float = 0.0, n: int = 512, h: float = 0.02, n_b: int = 157,
                      re: float = 100.0, dt: float = 0.005):
    return W.cylinder_stretched(n, h, n_b, re, dt, 0, alpha=alpha, solver=W.SOLVER_AMG_PCG)


def poisson_rhs(ctx, q, conv, lam):
    """Right-hand side of the next step's Poisson solve (state untouched)."""
    torch = ctx._torch
    ctx.stage_walls(q)
    r1, _ = ctx.stage_rhs1(q, conv)
    qs = q.clone()
    ctx.solve_velocity(r1, qs)
    return ctx.stage_rhs2(qs)


def harvest(alphas, steps_at, npairs, keep_every, log, **wl_kw):
    """(r1, e1) pairs (float32 CUDA tensors, one row per pair)."""
    import torch
    R1, E1, meta = [], [], []
    for a in alphas:
        wl = training_workload(alpha=a, **wl_kw)
        ctx = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-8)
        tight = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-12, poisson_maxit=20000)
        q, conv, lam = ctx.init_state()
        step = 0
        for target in steps_at:
            if target > step:
                ctx.step(q, conv, lam, target - step, stats=False)
                step = target
            rhs = poisson_rhs(ctx, q, conv, lam)
            xstar = lam.clone()
            tight.solve_poisson(rhs, xstar)
            x = lam.clone()
            r1, e1 = ctx.harvest(rhs, x, xstar, npairs)
            sel = torch.arange(0, r1.shape[0], keep_every, device=r1.device)
            R1.append(r1[sel].clone())
            E1.append(e1[sel].clone())
            meta.append({"alpha": a, "step": target, "pairs": int(sel.numel()),
                         "iterations_seen": int(r1.shape[0])})
            log(f"harvest alpha {a:+.4f} step {target}: {int(sel.numel())} pairs "
                f"of {int(r1.shape[0])} iterations")
            del r1, e1
        ctx.close()
        tight.close()
    return torch.cat(R1), torch.cat(E1), meta


def train(ctx, R1, E1, epochs, batch, lr, halve_at, seed, log):
    rng = np.random.default_rng(seed)
    S = R1.shape[0]
    losses = []
    for ep in range(epochs):
        cur_lr = lr * 0.5 ** sum(1 for e in halve_at if ep >= e)
        order = rng.permutation(S).astype(np.int32)
        t0 = time.time()
        L = ctx.nn_train(R1, E1, order, batch, cur_lr)
        losses.append(L)
        log(f"epoch {ep:3d} lr {cur_lr:.2e} loss {L:.5f} ({time.time() - t0:.1f} s)")
    return losses


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="weights file (.npy)")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--angles", type=int, default=6, help="number of inflow angles")
    ap.add_argument("--steps-at", default="2,6,15,30", help="time steps at which to harvest")
    ap.add_argument("--npairs", type=int, default=500)
    ap.add_argument("--keep-every", type=int, default=10)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    import torch
    rng = np.random.default_rng(args.seed)
    alphas = [float(a) for a in rng.uniform(-10.0, 10.0, size=args.angles) * math.pi / 180.0]
    steps_at = [int(s) for s in args.steps_at.split(",")]
    t0 = time.time()
    R1, E1, meta = harvest(alphas, steps_at, args.npairs, args.keep_every, log, n=args.n)
    t_h = time.time() - t0
    log(f"{R1.shape[0]} pairs of {R1.shape[1]} unknowns harvested in {t_h:.1f} s")
    ctx = ibpm.Context(training_workload(n=args.n), poisson_solver=1)
    ctx.nn_init(args.init_seed)
    halve_at = [int(args.epochs * 0.5), int(args.epochs * 0.75)]
    t1 = time.time()
    losses = train(ctx, R1, E1, args.epochs, args.batch, args.lr, halve_at, args.seed + 1, log)
    t_t = time.time() - t1
    w = ctx.nn_get_weights()
    np.save(args.out, w)
    rec = {"workload": training_workload(n=args.n).name, "alphas": alphas, "steps_at": steps_at,
           "npairs": args.npairs, "keep_every": args.keep_every, "pairs": int(R1.shape[0]),
           "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "halve_at": halve_at,
           "seed": args.seed, "init_seed": args.init_seed, "losses": losses,
           "harvest_s": t_h, "train_s": t_t, "per_solve": meta}
    with open(args.out.rsplit(".", 1)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    log(f"trained in {t_t:.1f} s; final loss {losses[-1]:.5f}; weights -> {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()
