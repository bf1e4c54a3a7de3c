"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs.

Bar (FP64): operators and stages agree to round-off (1e-12 relative to the
largest entry); solves and time steps run at a 1e-12 relative residual on
both sides agree to 1e-10 relative L2 in velocity and in lambda; the
smoothed-aggregation aggregates, being integer work, agree exactly."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W
from oracle import flow, solvers
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

TIGHT = 1e-12


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _maxrel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _walls_pack(w):
    return ibpm.pack_walls({k: getattr(w, k) for k in ("uL", "uR", "vB", "vT", "uBt", "uTt", "vLt", "vRt")})


WORKLOADS = {
    "tiny_stretched": lambda: W.tiny(16, 14, 8, 0.2, stretched=True, dt=0.02, nu=0.05),
    "cyl96": lambda: W.cylinder_small(96, 60),
    "cyl512": lambda: W.cylinder_512(),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_operators_match_oracle(name):
    wl = WORKLOADS[name]()
    print(f"[apply] {name}", flush=True)
    P = Problem(wl, poisson_solver=0)
    ctx = ibpm.Context(wl, poisson_solver=0)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(ctx.n_lambda)
    y = _n(ctx.apply_K(_t(x)))
    assert _maxrel(y, P.ops.K @ x) < 1e-13
    xq = rng.standard_normal(ctx.n_q)
    yq = _n(ctx.apply_A(_t(xq)))
    assert _maxrel(yq, P.ops.A @ xq) < 1e-13
    ctx.close()


def test_operator_dense_body():
    """A body with about four points per cell width: each cell couples to up
    to 36 force unknowns and each force row has up to 44 entries (against 9
    and 19 on the cylinder workloads); the operator must still match the
    oracle."""
    wl = W.cylinder_small(96, 300)
    print("[apply] cyl96 with 300 body points", flush=True)
    P = Problem(wl, poisson_solver=0)
    Kc = P.ops.K.tocsr()
    nc = wl.nx * wl.ny
    cols = [Kc.indices[Kc.indptr[i]:Kc.indptr[i + 1]] for i in range(nc)]
    assert max(int((c >= nc).sum()) for c in cols) > 10
    assert np.diff(Kc[nc:].tocsr().indptr).max() > 24
    ctx = ibpm.Context(wl, poisson_solver=0)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(ctx.n_lambda)
    y = _n(ctx.apply_K(_t(x)))
    assert _maxrel(y, P.ops.K @ x) < 1e-13
    ctx.close()


def test_operators_two_row_tiles_with_a_ragged_last_column():
    """A 1500^2 grid: the operators run in tiles of two rows (east / west
    values through LDS, one barrier per block) and the last tile of each
    row band is ragged (1500 = 5 x 256 + 220 cells, 1499 u faces), so lanes
    past the last column take the barrier without a column; K and A must
    still match the oracle on every row."""
    wl = W.cylinder_stretched(1500, 0.005, 628, 100.0, 0.002, 0)
    print("[apply] cylinder 1500^2", flush=True)
    P = Problem(wl, poisson_solver=0)
    ctx = ibpm.Context(wl, poisson_solver=0)
    rng = np.random.default_rng(13)
    x = rng.standard_normal(ctx.n_lambda)
    y = _n(ctx.apply_K(_t(x)))
    assert _maxrel(y, P.ops.K @ x) < 1e-13
    xq = rng.standard_normal(ctx.n_q)
    yq = _n(ctx.apply_A(_t(xq)))
    assert _maxrel(yq, P.ops.A @ xq) < 1e-13
    ctx.close()


def _oracle_state(P, steps):
    st = P.initial_state()
    for _ in range(steps):
        st, _ = P.step(st)
    return st


@pytest.mark.parametrize("name", ["tiny_stretched", "cyl96"])
def test_stages_match_oracle(name):
    wl = WORKLOADS[name]()
    print(f"[stages] {name}", flush=True)
    P = Problem(wl, poisson_solver=0, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    g, o = P.grid, P.ops
    st = _oracle_state(P, 2)
    ctx = ibpm.Context(wl, poisson_solver=0)
    ctx.set_walls(0, _walls_pack(st.walls))
    ctx.set_step(st.step)
    q = _t(st.q)
    # walls n -> n+1
    ctx.stage_walls(q)
    w1_ref = flow.update_walls(g, st.walls, st.q, wl.uinf, wl.alpha, o.dt)
    w1 = ctx.get_walls(1)
    assert _maxrel(w1, _walls_pack(w1_ref)) < 1e-13
    # momentum right-hand side and convection
    r1, conv_now = ctx.stage_rhs1(q, _t(st.conv_prev))
    conv_ref = flow.convection(g, st.q, st.walls)
    r1_ref = flow.momentum_rhs(o, st.q, conv_ref, st.conv_prev, st.walls, w1_ref)
    assert _maxrel(_n(conv_now), conv_ref) < 1e-12
    assert _maxrel(_n(r1), r1_ref) < 1e-12
    # Poisson right-hand side from the oracle's q*
    dinv = 1.0 / o.A.diagonal()
    qs, _, _ = solvers.pcg(o.apply_A, r1_ref, st.q, lambda r: dinv * r, TIGHT, 5000)
    rhs = _n(ctx.stage_rhs2(_t(qs)))
    rhs_ref = flow.poisson_rhs(o, qs, w1_ref, P.ub)
    assert _maxrel(rhs, rhs_ref) < 1e-12
    # projection and forces from the oracle's lambda
    lam, _, _ = P.solve_poisson(rhs_ref, st.lam, rtol=TIGHT, maxit=20000)
    qn = _n(ctx.stage_project(_t(qs), _t(lam)))
    assert _maxrel(qn, flow.project(o, qs, lam)) < 1e-13
    fx, fy = ctx.forces()
    fx_ref, fy_ref = flow.body_force(o, lam)
    assert abs(fx - fx_ref) <= 1e-12 * abs(fx_ref) + 1e-14
    assert abs(fy - fy_ref) <= 1e-12 * abs(fx_ref) + 1e-14
    # first step uses the current convection twice (AB2 start-up)
    ctx.set_step(0)
    r1b, _ = ctx.stage_rhs1(q, _t(np.full(g.n_q, 1e30)))
    r1b_ref = flow.momentum_rhs(o, st.q, conv_ref, conv_ref, st.walls, w1_ref)
    assert _maxrel(_n(r1b), r1b_ref) < 1e-12
    ctx.close()


@pytest.mark.parametrize("name", ["cyl96", "cyl512"])
def test_aggregates_match_oracle_exactly(name):
    wl = WORKLOADS[name]()
    print(f"[aggregates] {name}", flush=True)
    P = Problem(wl, poisson_solver=1)
    ctx = ibpm.Context(wl, poisson_solver=1)
    sizes, nnz = ctx.hierarchy()
    assert sizes == P.H.sizes()
    for l in range(len(sizes) - 1):
        np.testing.assert_array_equal(ctx.aggregates(l), P.H.levels[l].agg)
    ctx.close()


@pytest.mark.parametrize("solver", [0, 1])
def test_poisson_solve_matches_oracle(solver):
    wl = W.cylinder_small(96, 60)
    print(f"[poisson] solver {solver}", flush=True)
    P = Problem(wl, poisson_solver=solver, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    st = _oracle_state(P, 1)
    o = P.ops
    w1 = flow.update_walls(P.grid, st.walls, st.q, wl.uinf, wl.alpha, o.dt)
    conv = flow.convection(P.grid, st.q, st.walls)
    r1 = flow.momentum_rhs(o, st.q, conv, st.conv_prev, st.walls, w1)
    dinv = 1.0 / o.A.diagonal()
    qs, _, _ = solvers.pcg(o.apply_A, r1, st.q, lambda r: dinv * r, TIGHT, 5000)
    rhs = flow.poisson_rhs(o, qs, w1, P.ub)
    x0 = np.zeros_like(rhs)
    ref, it_ref, res_ref = P.solve_poisson(rhs, x0, rtol=TIGHT, maxit=50000)
    ctx = ibpm.Context(wl, poisson_solver=solver, poisson_rtol=TIGHT, poisson_maxit=50000)
    lam = _t(x0)
    s = ctx.solve_poisson(_t(rhs), lam)
    assert s["relres"] <= TIGHT * 1.01
    assert _rel(_n(lam), ref) < 1e-10
    # production tolerance: same algorithm, so the iteration counts agree
    ref8, it8, _ = P.solve_poisson(rhs, x0, rtol=1e-8)
    ctx8 = ibpm.Context(wl, poisson_solver=solver, poisson_rtol=1e-8)
    lam8 = _t(x0)
    s8 = ctx8.solve_poisson(_t(rhs), lam8)
    print(f"  iters gpu {s8['iters']} oracle {it8}; diff at 1e-8 {_rel(_n(lam8), ref8):.2e}")
    assert abs(s8["iters"] - it8) <= 2
    assert s8["relres"] <= 1e-8
    ctx.close()
    ctx8.close()


def test_velocity_solve_matches_oracle():
    wl = W.cylinder_512()
    P = Problem(wl, poisson_solver=0)
    o = P.ops
    rng = np.random.default_rng(3)
    b = o.A @ (rng.standard_normal(o.n_q))
    x0 = np.zeros_like(b)
    ref, it_ref, _ = solvers.jacobi_pcg(o.A, b, x0, TIGHT, 5000)
    ctx = ibpm.Context(wl, poisson_solver=0, vel_rtol=TIGHT)
    x = _t(x0)
    s = ctx.solve_velocity(_t(b), x)
    assert _rel(_n(x), ref) < 1e-10
    assert abs(s["iters"] - it_ref) <= 1
    ctx.close()


def _run_both(wl, steps, solver, rtol):
    ctx = ibpm.Context(wl, poisson_solver=solver, vel_rtol=rtol, poisson_rtol=rtol,
                       poisson_maxit=50000)
    q, conv, lam = ctx.init_state()
    gstats = [ctx.step(q, conv, lam, 1) for _ in range(steps)]
    P = Problem(wl, poisson_solver=solver, vel_rtol=rtol, poisson_rtol=rtol)
    P.wl = wl.replace(poisson_maxit=50000)
    st, infos = P.run(steps)
    R = P.grid.R_diag()
    eu = _rel(_n(q) / R, st.q / R)
    el = _rel(_n(lam), st.lam)
    ctx.close()
    return eu, el, gstats, infos


def test_trajectory_96_twenty_steps_jacobi():
    wl = W.cylinder_small(96, 60)
    eu, el, g, o = _run_both(wl, 20, 0, TIGHT)
    print(f"  96^2 x 20 steps: velocity {eu:.2e} lambda {el:.2e}; Fx {g[-1]['fx']:.12f} vs {o[-1].fx:.12f}")
    assert eu < 1e-10 and el < 1e-10
    assert abs(g[-1]["fx"] - o[-1].fx) < 1e-9 * abs(o[-1].fx)


def test_trajectory_96_amg_production_tolerance():
    """At the production tolerance the two runs follow the same iteration
    counts; differences are reported, the bar is the solver tolerance."""
    wl = W.cylinder_small(96, 60)
    eu, el, g, o = _run_both(wl, 10, 1, 1e-8)
    print(f"  96^2 x 10 steps at 1e-8: velocity {eu:.2e} lambda {el:.2e}")
    assert eu < 1e-7 and el < 1e-6
    its_g = [s["last_poisson_iters"] for s in g]
    its_o = [i.poisson_iters for i in o]
    assert max(abs(a - b) for a, b in zip(its_g, its_o)) <= 2


@pytest.mark.timeout(900)
def test_lambda_512_solve_at_the_fp64_floor():
    """One Poisson solve of the 512^2 trajectory (the second step's
    right-hand side and warm start, both from the oracle) against the exact
    solution of the oracle's system (sparse LU).  K is ill-conditioned
    (condition number ~1e9: its smallest eigenvalue belongs to the interior
    pressure / normal force mode), so two FP64 CG implementations stop at
    different points of an error floor: as the tolerance tightens past 1e-13
    the true residual of either levels off near 2.5e-14 and the error with it
    (the oracle's own AMG-PCG at 1e-11 of the exact solution, the GPU's at
    5e-11).  The GPU operator agrees with the oracle's to rounding on the
    exact solution, and the GPU solution lies within the 1e-10 bar of both
    the exact solution and the oracle's AMG-PCG solution."""
    import scipy.sparse.linalg as spla
    wl = W.cylinder_512()
    P = Problem(wl, poisson_solver=1, vel_rtol=1e-13, poisson_rtol=1e-13)
    rhs, st = _poisson_rhs_after(P, 1)
    o = P.ops
    exact = spla.splu(o.K.tocsc()).solve(rhs)
    ref, _, _ = P.solve_poisson(rhs, st.lam, rtol=1e-13, maxit=50000)
    ctx = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-13, poisson_maxit=5000)
    dK = _rel(_n(ctx.apply_K(_t(exact))), o.K @ exact)
    lam = _t(st.lam)
    s = ctx.solve_poisson(_t(rhs), lam)
    ctx.close()
    lg = _n(lam)
    print(f"  K on the exact solution: GPU vs oracle {dK:.2e}; GPU solve: relres {s['relres']:.2e}, "
          f"vs exact {_rel(lg, exact):.2e}, vs oracle AMG-PCG {_rel(lg, ref):.2e} "
          f"(oracle vs exact {_rel(ref, exact):.2e})", flush=True)
    assert dK < 1e-15
    assert s["relres"] <= 1.2e-13
    assert _rel(lg, exact) < 1e-10 and _rel(lg, ref) < 1e-10


@pytest.mark.timeout(900)
def test_trajectory_512_amg_ten_steps():
    """Ten steps of the 512^2 cylinder at a 1e-13 residual on both sides:
    velocity to the 1e-10 bar.  lambda is recomputed every step from the
    (well-determined) predicted velocity, so its difference stays at the
    FP64 floor of one ill-conditioned solve (see the test above: ~5e-11 of
    the exact solution per solve, the oracle's own floor 1e-11) times the
    spread of two implementations' stopping points, which is bounded here by
    5e-10; the GPU lambda is also checked by its backward error in the
    oracle's operator."""
    wl = W.cylinder_512()
    rtol = 1e-13
    eu, el, g, o = _run_both(wl, 10, 1, rtol)
    print(f"  512^2 x 10 steps AMG: velocity {eu:.2e} lambda {el:.2e}; Fx {g[-1]['fx']:.12f} vs "
          f"{o[-1].fx:.12f}; iters {[s['last_poisson_iters'] for s in g]} vs {[i.poisson_iters for i in o]}")
    assert eu < 1e-10 and el < 5e-10
    assert abs(g[-1]["fx"] - o[-1].fx) < 1e-10 * abs(o[-1].fx)
    # backward error of a GPU Poisson solve in the oracle's system, on the
    # GPU's own right-hand side of step 2
    P = Problem(wl, poisson_solver=1)
    ctx = ibpm.Context(wl, poisson_solver=1, vel_rtol=rtol, poisson_rtol=rtol, poisson_maxit=50000)
    q, conv, lam = ctx.init_state()
    ctx.step(q, conv, lam, 1)
    ctx.stage_walls(q)
    r1, _ = ctx.stage_rhs1(q, conv)
    qs = q.clone()
    ctx.solve_velocity(r1, qs)
    rhs = ctx.stage_rhs2(qs)
    s = ctx.solve_poisson(rhs, lam)
    rhs_h = _n(rhs)
    be = np.linalg.norm(rhs_h - P.ops.K @ _n(lam)) / np.linalg.norm(rhs_h)
    print(f"  backward error of the GPU lambda in the oracle system: {be:.2e} "
          f"(GPU true residual {s['relres']:.2e})")
    assert be < 10 * rtol
    ctx.close()


def test_uniform_flow_without_body_stays_uniform():
    wl = W.tiny(16, 14, 0, stretched=True).replace(alpha=0.2)
    ctx = ibpm.Context(wl, poisson_solver=0, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    q, conv, lam = ctx.init_state()
    q0 = _n(q).copy()
    ctx.step(q, conv, lam, 3)
    assert np.abs(_n(q) - q0).max() < 1e-13
    assert np.abs(_n(lam)).max() < 1e-12
    ctx.close()


def test_solver_edge_cases():
    wl = W.cylinder_small(48, 30)
    ctx = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-8, poisson_maxit=3)
    n = ctx.n_lambda
    # zero right-hand side: zero solution, no iterations
    lam = _t(np.ones(n))
    s = ctx.solve_poisson(_t(np.zeros(n)), lam)
    assert s["iters"] == 0 and np.all(_n(lam) == 0.0)
    # iteration limit
    rhs = np.random.default_rng(1).standard_normal(n)
    rhs[0] = 0.0
    lam = _t(np.zeros(n))
    with pytest.raises(ibpm.IBPMError) as e:
        ctx.solve_poisson(_t(rhs), lam)
    assert e.value.code == ibpm.IBPM_ENOTCONV
    s = ctx.solve_poisson(_t(rhs), _t(np.zeros(n)), allow_fail=True)
    assert s["iters"] == 3 and s["status"] == ibpm.IBPM_ENOTCONV and s["relres"] > 1e-8
    # NaN in the right-hand side
    bad = rhs.copy()
    bad[5] = np.nan
    with pytest.raises(ibpm.IBPMError) as e:
        ctx.solve_poisson(_t(bad), _t(np.zeros(n)))
    assert e.value.code == ibpm.IBPM_ENAN
    # already converged initial guess: zero iterations
    ctx2 = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-6)
    x = _t(np.zeros(n))
    ctx2.solve_poisson(_t(rhs), x)
    s = ctx2.solve_poisson(_t(rhs), x)
    assert s["iters"] == 0
    # wrong tensor types are refused by the binding
    with pytest.raises(TypeError):
        ctx2.solve_poisson(torch.zeros(n, dtype=torch.float32, device="cuda"), x)
    ctx.close()
    ctx2.close()


def test_runs_are_bitwise_deterministic():
    wl = W.cylinder_small(96, 60)
    outs = []
    for _ in range(2):
        ctx = ibpm.Context(wl, poisson_solver=1)
        q, conv, lam = ctx.init_state()
        ctx.step(q, conv, lam, 3)
        outs.append((_n(q).copy(), _n(lam).copy()))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.timeout(600)
def test_full_size_2048_operators_and_stages():
    """Largest workload (2048^2, 4.2M cells, 628 points) in the launch
    configuration of the time step: the Poisson operator, the velocity
    operator and the right-hand-side stages against the oracle on every
    row."""
    wl = W.cylinder_2048()
    print("[2048] oracle assembly", flush=True)
    P = Problem(wl, poisson_solver=0)
    g, o = P.grid, P.ops
    ctx = ibpm.Context(wl, poisson_solver=0)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(ctx.n_lambda)
    assert _maxrel(_n(ctx.apply_K(_t(x))), o.K @ x) < 1e-13
    xq = rng.standard_normal(ctx.n_q)
    assert _maxrel(_n(ctx.apply_A(_t(xq))), o.A @ xq) < 1e-13
    # a perturbed freestream state
    st = P.initial_state()
    qn = st.q * (1.0 + 0.05 * rng.standard_normal(g.n_q))
    conv_prev = flow.convection(g, st.q, st.walls)
    ctx.set_step(3)
    q = _t(qn)
    ctx.stage_walls(q)
    w1 = flow.update_walls(g, st.walls, qn, wl.uinf, wl.alpha, o.dt)
    r1, conv_now = ctx.stage_rhs1(q, _t(conv_prev))
    conv_ref = flow.convection(g, qn, st.walls)
    assert _maxrel(_n(conv_now), conv_ref) < 1e-12
    assert _maxrel(_n(r1), flow.momentum_rhs(o, qn, conv_ref, conv_prev, st.walls, w1)) < 1e-12
    rhs = _n(ctx.stage_rhs2(q))
    assert _maxrel(rhs, flow.poisson_rhs(o, qn, w1, P.ub)) < 1e-12
    lam = rng.standard_normal(ctx.n_lambda)
    assert _maxrel(_n(ctx.stage_project(q, _t(lam))), flow.project(o, qn, lam)) < 1e-13
    ctx.close()


def _poisson_rhs_after(P, steps):
    st = _oracle_state(P, steps)
    o = P.ops
    w1 = flow.update_walls(P.grid, st.walls, st.q, P.wl.uinf, P.wl.alpha, o.dt)
    conv = flow.convection(P.grid, st.q, st.walls)
    r1 = flow.momentum_rhs(o, st.q, conv, st.conv_prev, st.walls, w1)
    dinv = 1.0 / o.A.diagonal()
    qs, _, _ = solvers.pcg(o.apply_A, r1, st.q, lambda r: dinv * r, TIGHT, 5000)
    return flow.poisson_rhs(o, qs, w1, P.ub), st


@pytest.mark.timeout(600)
def test_mixed_precision_poisson_solve_against_fp64_oracle():
    """FP32 inner AMG-PCG in FP64 refinement: the true FP64 residual meets
    1e-8 and the solution is within the FP64 oracle's 1e-8 spread."""
    wl = W.cylinder_512()
    P = Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    rhs, st = _poisson_rhs_after(P, 1)
    ref, _, _ = P.solve_poisson(rhs, st.lam, rtol=TIGHT, maxit=50000)
    ctx = ibpm.Context(wl, poisson_solver=2, poisson_rtol=1e-8)
    lam = _t(st.lam)
    s = ctx.solve_poisson(_t(rhs), lam)
    e = _rel(_n(lam), ref)
    ctx64 = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-8)
    lam64 = _t(st.lam)
    s64 = ctx64.solve_poisson(_t(rhs), lam64)
    e64 = _rel(_n(lam64), ref)
    # the velocity field the solve produces: q = q* - B^1 Q lambda
    o = P.ops
    R = P.grid.R_diag()   # the projection is linear in lambda: compare B^1 Q lambda
    du = _rel(o.B1 * (o.Q @ _n(lam)) / R, o.B1 * (o.Q @ ref) / R)
    du64 = _rel(o.B1 * (o.Q @ _n(lam64)) / R, o.B1 * (o.Q @ ref) / R)
    print(f"  mixed: {s['iters']} inner / {s['outer_iters']} outer, relres {s['relres']:.2e}, "
          f"lambda err {e:.2e}, projection err {du:.2e}; fp64: {s64['iters']} iters, "
          f"lambda err {e64:.2e}, projection err {du64:.2e}")
    assert s["relres"] <= 1e-8 and s["outer_iters"] >= 1
    # lambda carries the ill-conditioned interior-pressure / force modes; the
    # velocity correction it produces is the field the step uses.  A 1e-8
    # residual bounds that error only through the conditioning of K, so the
    # bar is the FP64 solver's own error at the same stopping test
    assert du < max(3.0 * du64, 1e-7)
    assert e < 1e-4
    # refinement carries the FP32 inner solves past FP32 accuracy: at a 1e-11
    # stopping test the projection error drops well below its 1e-8 value
    ctx.close()
    ctx = ibpm.Context(wl, poisson_solver=2, poisson_rtol=1e-11, poisson_maxit=20000)
    lam = _t(st.lam)
    s2 = ctx.solve_poisson(_t(rhs), lam)
    du2 = _rel(o.B1 * (o.Q @ _n(lam)) / R, o.B1 * (o.Q @ ref) / R)
    print(f"  mixed at 1e-11: {s2['iters']} inner / {s2['outer_iters']} outer, projection err {du2:.2e}")
    assert s2["relres"] <= 1e-11 and du2 < 5e-9 and du2 < du / 20
    ctx.close()
    ctx64.close()


def test_mixed_precision_trajectory_velocity_and_drag():
    wl = W.cylinder_small(96, 60).replace(poisson_solver=2)
    ctx = ibpm.Context(wl, poisson_solver=2, poisson_rtol=1e-8)
    q, conv, lam = ctx.init_state()
    for _ in range(10):
        sm = ctx.step(q, conv, lam, 1)
    P = Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    ost, infos = P.run(10)
    R = P.grid.R_diag()
    eu = _rel(_n(q) / R, ost.q / R)
    ecd = abs(sm["fx"] - infos[-1].fx) / abs(infos[-1].fx)
    print(f"  96^2 mixed x 10 steps: velocity err {eu:.2e}, Cd err {ecd:.2e}")
    assert eu < 1e-7 and ecd < 1e-6
    ctx.close()


def test_graph_replay_matches_eager_launches():
    """CG iterations replayed as HIP graphs give bitwise the results of the
    same launches made one by one, over repeated solves (the graph is reused)
    with eager work in between, for the velocity, Poisson FP64 and inner FP32
    solves."""
    wl = W.cylinder_small(96, 60).replace(poisson_solver=1)
    out = {}
    for graphs in (0, 1):
        for solver in (1, 2):
            ctx = ibpm.Context(wl, poisson_solver=solver, use_graphs=graphs)
            q, conv, lam = ctx.init_state()
            stats = []
            for _ in range(3):
                stats.append(ctx.step(q, conv, lam, 1))
                _ = ctx.apply_K(lam)          # eager work between the replays
            out[(graphs, solver)] = (_n(q).copy(), _n(lam).copy(),
                                     [s["poisson_iters"] for s in stats])
            ctx.close()
    for solver in (1, 2):
        a, b = out[(0, solver)], out[(1, solver)]
        print(f"  solver {solver}: iterations eager {a[2]} graph {b[2]}")
        assert a[2] == b[2]
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def test_fused_transfers_match_separate_kernels():
    """The V-cycle with the residual folded into the restriction and the
    prolongation folded into the first post-sweep (products R A and A P)
    against the same cycle with separate kernels (the form of the large
    grids), both against the oracle on the 512^2 grid, where every level
    takes the fused form: the 1e-13 solves agree with the oracle (the
    projection term B Q lambda to 1e-11, 4e-13 measured; true residual at
    the tolerance), and at 1e-8 both take the oracle's iteration count to
    within 2."""
    wl = W.cylinder_512()
    P = Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=1e-13)
    rhs, st = _poisson_rhs_after(P, 1)
    ref, _, _ = P.solve_poisson(rhs, st.lam, rtol=1e-13, maxit=50000)
    _, it8, _ = P.solve_poisson(rhs, st.lam, rtol=1e-8)
    o = P.ops
    R = P.grid.R_diag()
    proj_ref = o.B1 * (o.Q @ ref) / R
    for fuse in (1, 0):
        print(f"[poisson 512] fuse_transfers {fuse}", flush=True)
        ctx = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-13, poisson_maxit=50000, fuse_transfers=fuse)
        lam = _t(st.lam)
        s = ctx.solve_poisson(_t(rhs), lam)
        d = _rel(o.B1 * (o.Q @ _n(lam)) / R, proj_ref)
        ctx.close()
        ctx8 = ibpm.Context(wl, poisson_solver=1, poisson_rtol=1e-8, fuse_transfers=fuse)
        lam8 = _t(st.lam)
        s8 = ctx8.solve_poisson(_t(rhs), lam8)
        ctx8.close()
        print(f"  1e-13: relres {s['relres']:.2e}, projection diff {d:.2e}; 1e-8: iters {s8['iters']} "
              f"(oracle {it8})")
        # CG stops on its recursively updated residual; the true residual
        # recomputed at exit drifts from it by rounding over ~260 iterations
        # (the oracle's own solve of the second step ends at 1.05e-13)
        assert s["relres"] <= 1e-13 * 1.2
        assert d < 1e-11
        assert abs(s8["iters"] - it8) <= 2


def test_amg_solve_1024_with_one_block_finalizes():
    """The 1024^2 grid (1,049,204 unknowns): the level-0 walker has about
    4,100 blocks, more partials than the product and update kernels sum
    themselves, so every iteration ends with one-block finalizes (no
    deferred stop test), and level 0 keeps the separate residual and
    restriction (more than 600,000 unknowns).  FP64 AMG-PCG and the FP32
    V-cycle solver on a seeded right-hand side: the solution solves the
    oracle's system, ||b - K lambda|| within the tolerance with the oracle's
    K, at rtol 1e-8 and 1e-11.  CG stops on its recursive residual and the
    true residual is recomputed at exit; at 1e-8 it meets the tolerance, at
    1e-11 (about 1,500 iterations) the two drift apart by some tens of per
    cent (1.23e-11 measured), so the bound there is 1.5 rtol.  (The oracle's
    own solve at this size takes minutes; the iteration counts are compared
    with the oracle's on the 96^2 and 512^2 grids.)"""
    wl = W.cylinder_1024()
    print("[poisson 1024] oracle operators", flush=True)
    P = Problem(wl, poisson_solver=0)
    K = P.ops.K.tocsr()
    rhs = np.random.default_rng(14).standard_normal(K.shape[0])
    rhs[0] = 0.0
    for solver in (1, 5, 2):
        for rtol in (1e-8, 1e-11):
            print(f"[poisson 1024] solver {solver} rtol {rtol:g}", flush=True)
            ctx = ibpm.Context(wl, poisson_solver=solver, poisson_rtol=rtol, poisson_maxit=20000)
            lam = _t(np.zeros(K.shape[0]))
            s = ctx.solve_poisson(_t(rhs), lam)
            ctx.close()
            back = np.linalg.norm(rhs - K @ _n(lam)) / np.linalg.norm(rhs)
            print(f"  iters {s['iters']}, relres {s['relres']:.2e}, backward error in the oracle's system {back:.2e}")
            # the refinement (solver 2) stops on the FP64 outer residual itself
            bound = rtol if (rtol >= 1e-8 or solver == 2) else 1.5 * rtol
            assert s["relres"] <= bound
            assert back <= 1.01 * bound


def test_fp32_cycle_solver_matches_fp64():
    """FP64 CG with the V-cycle in FP32 (a fixed linear preconditioner): the
    same 1e-8 true residual, the projected velocity within the FP64 solver's
    own error, and about the FP64 iteration count."""
    wl = W.cylinder_512()
    P = Problem(wl, poisson_solver=1, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    rhs, st = _poisson_rhs_after(P, 1)
    ref, _, _ = P.solve_poisson(rhs, st.lam, rtol=TIGHT, maxit=50000)
    o = P.ops
    R = P.grid.R_diag()
    out = {}
    for solver in (1, 5):
        ctx = ibpm.Context(wl, poisson_solver=solver, poisson_rtol=1e-8)
        lam = _t(st.lam)
        s = ctx.solve_poisson(_t(rhs), lam)
        out[solver] = (s, _rel(o.B1 * (o.Q @ _n(lam)) / R, o.B1 * (o.Q @ ref) / R))
        ctx.close()
    (s1, d1), (s5, d5) = out[1], out[5]
    print(f"  FP64 cycle {s1['iters']} iters, projection err {d1:.2e}; "
          f"FP32 cycle {s5['iters']} iters, projection err {d5:.2e}")
    assert s5["relres"] <= 1e-8
    assert d5 < max(3.0 * d1, 1e-7)
    assert s5["iters"] <= 1.2 * s1["iters"]


def test_pin_cell_and_dirichlet_walls_match_oracle():
    """A pinned cell other than cell 0 (here inside the coupling box of the
    body, next to coupled cells) and Dirichlet walls on all four sides: the
    operator on every row, and three time steps at a 1e-12 residual, against
    the oracle with the same parameters."""
    wl = W.cylinder_small(96, 60)
    pin = 48 * 96 + 60
    print("[pin/walls] cyl96 pin", pin, flush=True)
    wl = wl.replace(pin_cell=pin, bc_kind=(0, 0, 0, 0), bc_u=(1.0, 1.0, 1.0, 1.0),
                    bc_v=(0.1, 0.1, 0.0, 0.0))
    P = Problem(wl, poisson_solver=0, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    ctx = ibpm.Context(wl, poisson_solver=0, vel_rtol=TIGHT, poisson_rtol=TIGHT,
                       poisson_maxit=20000)
    rng = np.random.default_rng(17)
    x = rng.standard_normal(ctx.n_lambda)
    assert _maxrel(_n(ctx.apply_K(_t(x))), P.ops.K @ x) < 1e-13
    q, conv, lam = ctx.init_state()
    for _ in range(3):
        ctx.step(q, conv, lam, 1)
    st, _ = P.run(3)
    R = P.grid.R_diag()
    eu = _rel(_n(q) / R, st.q / R)
    el = _rel(_n(lam), st.lam)
    print(f"  velocity {eu:.2e} lambda {el:.2e}", flush=True)
    assert eu < 1e-10 and el < 1e-10
    assert _n(lam)[pin] == 0.0
    w = ibpm.unpack_walls(ctx.get_walls(1), wl.nx, wl.ny)
    assert np.all(w["uR"] == 1.0) and np.all(w["vLt"] == 0.1) and np.all(w["vB"] == 0.0)
    ctx.close()
