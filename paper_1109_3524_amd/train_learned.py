"""Train the correction network of the learned preconditioner stage on the
device.

Recipe (all seeded):
  1. Variants of the training flow are drawn: the cylinder's centre uniform
     in [-0.46, 0.46]^2 (the body and its delta supports stay inside the
     uniform patch of the grid) and the inflow angle uniform in +-10 degrees.
     Each variant has a context of its own -- its own E, K and hierarchy,
     and the delta weights that carry the force residuals to the network's
     cell grid -- and its flow is started impulsively.
  2. At a few time steps of each run the right-hand side of the modified
     Poisson system (Eq. 11b) is formed with the library's stages, solved to
     a 1e-12 relative residual (x*), and an AMG-PCG solve from the previous
     lambda is replayed with ibpm_harvest, which stores before each iteration
     the residual left by one V-cycle, r1 = r - K V(r), and the error that
     remains, e1 = x* - x - V(r).  Up to `per_solve` pairs spread evenly over
     the iterations are kept.
  3. The network is trained with Adam on the energy-norm loss (the share of
     the error that the optimally scaled correction removes).  A batch holds
     pairs of one variant: that variant's context computes each pair's loss
     and gradient with the current weights (ibpm_nn_loss_grad, its own K in
     the loss), and one Adam step on the summed gradient runs on the master
     weights (ibpm_nn_adam_step).  The batches are drawn anew and shuffled
     each epoch by a seeded generator, the learning rate halved at fixed
     epochs; training stops early, after a whole batch, when a time budget is
     spent.

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

CENTRE_RANGE = 0.46      # |cx|, |cy| of the body centre
ANGLE_RANGE = 10.0       # inflow angle, degrees


def training_workload(alpha: float = 0.0, cx: float = 0.0, cy: float = 0.0, n: int = 512, h: float = 0.02,
                      n_b: int = 157, re: float = 100.0, dt: float = 0.005):
    return W.cylinder_stretched(n, h, n_b, re, dt, 0, cx=cx, cy=cy, alpha=alpha, solver=W.SOLVER_AMG_PCG)


def draw_variants(count: int, seed: int):
    """(cx, cy, alpha) of each training flow."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(-CENTRE_RANGE, CENTRE_RANGE, size=count)
    cy = rng.uniform(-CENTRE_RANGE, CENTRE_RANGE, size=count)
    al = rng.uniform(-ANGLE_RANGE, ANGLE_RANGE, size=count) * math.pi / 180.0
    return [(float(a), float(b), float(c)) for a, b, c in zip(cx, cy, al)]


def poisson_rhs(ctx, q, conv, lam):
    """Right-hand side of the next step's Poisson solve (state untouched)."""
    ctx.stage_walls(q)
    r1, _ = ctx.stage_rhs1(q, conv)
    qs = q.clone()
    ctx.solve_velocity(r1, qs)
    return ctx.stage_rhs2(qs)


def harvest_variant(var, steps_at, npairs, per_solve, log, n=512):
    """The variant's context (kept for training) and its (r1, e1) pairs
    (float32 CUDA tensors, one row per pair)."""
    import torch
    cx, cy, a = var
    wl = training_workload(alpha=a, cx=cx, cy=cy, n=n)
    ctx = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-8)
    tight = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-12, poisson_maxit=20000)
    q, conv, lam = ctx.init_state()
    R1, E1, meta = [], [], []
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
        m = r1.shape[0]
        k = min(per_solve, m)
        sel = torch.unique(torch.linspace(0, m - 1, k, device=r1.device).round().long())
        R1.append(r1[sel].clone())
        E1.append(e1[sel].clone())
        meta.append({"cx": cx, "cy": cy, "alpha": a, "step": target, "pairs": int(sel.numel()),
                     "iterations_seen": int(m)})
        del r1, e1
    tight.close()
    R1, E1 = torch.cat(R1), torch.cat(E1)
    log(f"variant centre ({cx:+.3f}, {cy:+.3f}) angle {a * 180 / math.pi:+.2f} deg: {R1.shape[0]} pairs")
    return ctx, R1, E1, meta


def train(master, ctxs, R1s, E1s, epochs, batch, lr, halve_at, seed, budget_s, log):
    """Adam on batches of one variant each (see the recipe); returns the mean
    loss of each epoch (the last one possibly cut by the time budget) and the
    batches done."""
    rng = np.random.default_rng(seed)
    t_start = time.time()
    losses, done = [], 0
    for ep in range(epochs):
        cur_lr = lr * 0.5 ** sum(1 for e in halve_at if ep >= e)
        batches = []
        for v, R in enumerate(R1s):
            perm = rng.permutation(R.shape[0])
            batches += [(v, perm[b0:b0 + batch]) for b0 in range(0, len(perm), batch)]
        order = rng.permutation(len(batches))
        t0 = time.time()
        tot, cnt, stop = 0.0, 0, False
        for bi in order:
            v, idx = batches[bi]
            ctxs[v].nn_set_weights(master.nn_get_weights())
            g = np.zeros(ibpm.NN_PARAMS, dtype=np.float64)
            for i in idx:
                loss, gi = ctxs[v].nn_loss_grad(R1s[v][int(i)], E1s[v][int(i)])
                g += gi
                tot += loss
                cnt += 1
            master.nn_adam_step(g.astype(np.float32), cur_lr)
            done += 1
            if time.time() - t_start > budget_s:
                stop = True
                break
        losses.append(tot / max(cnt, 1))
        log(f"epoch {ep:3d} lr {cur_lr:.2e} loss {losses[-1]:.5f} over {cnt} pairs ({time.time() - t0:.1f} s)")
        if stop:
            log(f"time budget of {budget_s:.0f} s spent after {done} batches")
            break
    return losses, done


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True, help="weights file (.npy)")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--variants", type=int, default=40, help="training flows (body centre, inflow angle)")
    ap.add_argument("--steps-at", default="5,20,35,50", help="time steps at which to harvest")
    ap.add_argument("--npairs", type=int, default=500, help="iterations a harvest records at most")
    ap.add_argument("--per-solve", type=int, default=125, help="pairs kept per harvested solve")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--init-seed", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--budget-min", type=float, default=1e9, help="training time budget (minutes)")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    variants = draw_variants(args.variants, args.seed)
    steps_at = [int(s) for s in args.steps_at.split(",")]
    t0 = time.time()
    ctxs, R1s, E1s, meta = [], [], [], []
    for var in variants:
        c, r, e, m = harvest_variant(var, steps_at, args.npairs, args.per_solve, log, n=args.n)
        ctxs.append(c)
        R1s.append(r)
        E1s.append(e)
        meta += m
    t_h = time.time() - t0
    npairs = sum(int(r.shape[0]) for r in R1s)
    log(f"{npairs} pairs from {len(variants)} flows ({len(variants) * steps_at[-1]} time steps) "
        f"harvested in {t_h:.1f} s")
    for c in ctxs:
        c.nn_init(args.init_seed)
    master = ctxs[0]
    halve_at = [int(args.epochs * 0.5), int(args.epochs * 0.75)]
    t1 = time.time()
    losses, nbatches = train(master, ctxs, R1s, E1s, args.epochs, args.batch, args.lr, halve_at,
                             args.seed + 1, 60.0 * args.budget_min, log)
    t_t = time.time() - t1
    w = master.nn_get_weights()
    np.save(args.out, w)
    rec = {"workload": training_workload(n=args.n).name, "variants": variants,
           "centre_range": CENTRE_RANGE, "angle_range_deg": ANGLE_RANGE, "steps_at": steps_at,
           "npairs": args.npairs, "per_solve": args.per_solve, "pairs": npairs,
           "epochs_requested": args.epochs, "epochs_run": len(losses), "batches": nbatches,
           "batch": args.batch, "lr": args.lr, "halve_at": halve_at, "seed": args.seed,
           "init_seed": args.init_seed, "losses": losses, "harvest_s": t_h, "train_s": t_t,
           "per_solve_record": meta}
    with open(args.out.rsplit(".", 1)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    log(f"trained in {t_t:.1f} s; last epoch loss {losses[-1]:.5f}; weights -> {args.out}")
    for c in ctxs:
        c.close()


if __name__ == "__main__":
    main()
