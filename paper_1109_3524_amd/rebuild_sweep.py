"""Time steps of a heaving cylinder with the AMG hierarchy formed anew every
n moves (Sec. 4: the smoothed-aggregation hierarchy is re-used over several
steps of a moving body, since forming it costs more than it saves when done
at every step).

    python -m paper_1109_3524_amd.rebuild_sweep --grid 1024 --steps 40 --every 0,1,2,3,5

For each n: the body is moved before every step to its position at the time
the step advances to (E and K formed anew on the device), the hierarchy is
formed anew at every n-th move (0: never), and the mean wall time of a move
and of a step, the Poisson iterations per step and the hierarchies formed
are printed, one JSON line per n.
"""
from __future__ import annotations

import argparse
import json
import time

from . import ibpm
from . import workloads as W


def run(grid: int, steps: int, warmup: int, every: int) -> dict:
    import torch
    wl = W.heaving_cylinder(grid)
    ctx = ibpm.Context(wl, poisson_solver=W.SOLVER_AMG_PCG, moving_body=1, amg_rebuild_every=every)
    q, conv, lam = ctx.init_state()
    move_ms = step_ms = 0.0
    iters = 0
    refresh0 = 0
    for n in range(warmup + steps):
        if n == warmup:
            refresh0 = ctx.moving_info()["refreshes"]
        body = W.heave(wl, (n + 1) * wl.dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.move_body(*body)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s = ctx.step(q, conv, lam, 1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if n >= warmup:
            move_ms += 1e3 * (t1 - t0)
            step_ms += 1e3 * (t2 - t1)
            iters += s["poisson_iters"]
    info = ctx.moving_info()
    ctx.close()
    return {"grid": f"{grid}x{grid}", "nb": wl.nb, "rebuild_every": every, "steps": steps,
            "move_ms": move_ms / steps, "step_ms": step_ms / steps,
            "total_ms": (move_ms + step_ms) / steps, "poisson_iters": iters / steps,
            "refreshes": info["refreshes"] - refresh0}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--grid", type=int, default=1024, choices=(512, 1024, 2048))
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--every", default="0,1,2,3,5")
    a = ap.parse_args(argv)
    for every in (int(x) for x in a.every.split(",")):
        print(json.dumps(run(a.grid, a.steps, a.warmup, every)), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
