"""The level-0 prolongation and both post-smoothing sweeps in one pass
(strips with recomputed edges, plus three small passes over the box coupled
to the forces) against the three separate passes it replaces (the V-cycle of
Sec. 3, post = 2).

Every cell of z is formed by the same arithmetic in either form, so one
V-cycle (the first pair ibpm_harvest records, e1 = -V(r) for x = x* = 0) must
agree bit for bit; whole solves differ only through the order in which the
r . z partials are added, so their iteration counts agree and the solutions
within 1e-12.  Cases: the stretched 512^2 cylinder; a ragged 300 x 220 grid
(strips and blocks cut by both grid edges); a body near the pinned corner
(the box clipped by two walls, the pinned cell inside it); no body.  Each at
strip depths 8, 16 and 32; the FP32 cycle (result widened to FP64), the FP64
refinement around FP32 AMG-PCG and the flexible CG of the learned stage (no
r . z) too."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W

pytestmark = pytest.mark.gpu


def _uniform(nx, ny, lx, ly, n_b, cx=0.0, cy=0.0, radius=0.5):
    xf = W.uniform_faces(nx, -lx, lx)
    yf = W.uniform_faces(ny, -ly, ly)
    if n_b > 0:
        xb, yb = W.circle_points(n_b, cx, cy, radius)
    else:
        xb, yb = np.zeros(0), np.zeros(0)
    return W.Workload(name=f"uniform_{nx}x{ny}_{n_b}", xf=xf, yf=yf, xb=xb, yb=yb, ubx=np.zeros(n_b),
                      uby=np.zeros(n_b), nu=0.025, dt=0.01, nsteps=2, poisson_solver=W.SOLVER_AMG_PCG)


CASES = {
    "cylinder_512": lambda: W.cylinder_stretched(512, 0.02, 157, 40.0, 0.005, 2),
    "ragged_300x220": lambda: _uniform(300, 220, 2.0, 1.5, 80),
    "corner_body": lambda: _uniform(160, 128, 2.0, 1.6, 60, cx=-1.5, cy=-1.14, radius=0.4),
    "no_body": lambda: _uniform(192, 136, 2.0, 1.5, 0),
}


class _env:
    """IBPM_POST_FUSE / IBPM_POST_ROWS for the calls made inside."""

    def __init__(self, fuse, rows=None):
        self.kv = {"IBPM_POST_FUSE": str(fuse)}
        if rows:
            self.kv["IBPM_POST_ROWS"] = str(rows)

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in ("IBPM_POST_FUSE", "IBPM_POST_ROWS")}
        for k in self.old:
            os.environ.pop(k, None)
        os.environ.update(self.kv)

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _rhs(ctx, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(ctx.n_lambda)
    nc = ctx.nx * ctx.ny
    b[:nc] -= b[:nc].mean()
    b[ctx.wl.pin_cell] = 0.0
    return torch.as_tensor(b, dtype=torch.float64, device="cuda")


def _run(wl, fuse, rows, solver, seed=3):
    """One V-cycle (e1 of the first harvested pair) and one solve."""
    with _env(fuse, rows):
        ctx = ibpm.Context(wl, poisson_solver=solver, poisson_rtol=1e-12, poisson_maxit=3000)
        try:
            rhs = _rhs(ctx, seed)
            e1 = None
            if solver == W.SOLVER_AMG_PCG:
                z0 = ctx.zeros_lambda()
                _, e = ctx.harvest(rhs, z0, ctx.zeros_lambda(), 1)
                e1 = e[0].cpu().numpy()
            if solver == W.SOLVER_AMG_FCG_LEARNED:
                ctx.nn_init(5)
            lam = ctx.zeros_lambda()
            st = ctx.solve_poisson(rhs, lam)
            torch.cuda.synchronize()
            return e1, lam.cpu().numpy(), st
        finally:
            ctx.close()


@pytest.mark.parametrize("rows", [8, 16, 32])
@pytest.mark.parametrize("case", list(CASES))
def test_fused_post_smoothing_matches_separate_passes(case, rows):
    wl = CASES[case]()
    print(f"[post fuse] {case} ({wl.nx}x{wl.ny}, {wl.nb} points) rows {rows}", flush=True)
    e_off, l_off, s_off = _run(wl, 0, None, W.SOLVER_AMG_PCG)
    e_on, l_on, s_on = _run(wl, 1, rows, W.SOLVER_AMG_PCG)
    same = int(np.sum(e_on.view(np.uint32) != e_off.view(np.uint32)))
    dl = float(np.linalg.norm(l_on - l_off) / np.linalg.norm(l_off))
    print(f"  V-cycle entries differing: {same} of {e_on.size}; solve {s_on['iters']} vs {s_off['iters']} "
          f"iterations, lambda {dl:.2e}", flush=True)
    assert same == 0
    assert s_on["iters"] == s_off["iters"] and s_on["status"] == 0
    assert dl < 1e-12


@pytest.mark.parametrize("solver", [W.SOLVER_AMG_PCG_FP32_CYCLE, W.SOLVER_AMG_PCG_MIXED,
                                    W.SOLVER_AMG_FCG_LEARNED])
def test_fused_post_smoothing_in_the_other_solvers(solver):
    wl = CASES["ragged_300x220"]()
    print(f"[post fuse] solver {solver}", flush=True)
    _, l_off, s_off = _run(wl, 0, None, solver)
    _, l_on, s_on = _run(wl, 1, 16, solver)
    dl = float(np.linalg.norm(l_on - l_off) / np.linalg.norm(l_off))
    print(f"  {s_on['iters']} vs {s_off['iters']} iterations, lambda {dl:.2e}", flush=True)
    assert s_on["status"] == 0 and s_off["status"] == 0
    if solver == W.SOLVER_AMG_PCG_MIXED:
        # FP32 inner solves restarted by an FP64 refinement near FP32's
        # limit: the partial sums' order moves where each inner solve stops
        assert abs(s_on["iters"] - s_off["iters"]) <= 0.1 * s_off["iters"]
    else:
        assert abs(s_on["iters"] - s_off["iters"]) <= 1
    assert dl < 1e-10

