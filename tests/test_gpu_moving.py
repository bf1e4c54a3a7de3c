"""A body in prescribed motion on the GPU (Sec. 6, with the per-step update
of the forcing rows and the re-used hierarchy of Sec. 4): the operator K
re-assembled on the device after each move against the oracle's K at the
same positions (every stored entry), the stages that use E, trajectories of
a heaving cylinder against the oracle's moving-body steps, the hierarchy
formed anew on the device against the oracle's refresh on the same
aggregates, and the changed rows of K on the 2048^2 grid against the
products E B^1 G and E B^1 E^T formed from the oracle's pieces.

Bars: operator entries within 1e-13 of the largest entry; stages within
1e-12 (relative, element-wise maximum); trajectories to the 1e-10 bar on
velocity and lambda at a 1e-12 residual (as for the fixed body)."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W
from oracle import delta, flow, operators
from oracle.grid import Grid
from oracle.problem import Problem

pytestmark = pytest.mark.gpu

TIGHT = 1e-12


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _kdiff(Kg, Ko):
    D = (Kg - Ko).tocsr()
    scale = np.max(np.abs(Ko.data))
    return (np.max(np.abs(D.data)) / scale) if D.nnz else 0.0


CASES = {
    "tiny_stretched": lambda: W.tiny(16, 14, 6, 0.2, stretched=True),
    "cyl96": lambda: W.cylinder_small(96, 60),
}

# point offsets in cells (x, y) of successive moves
SHIFTS = [(0.31, -0.17), (0.83, 0.42), (-0.61, 0.55), (0.0, 0.0)]


@pytest.mark.parametrize("name", list(CASES))
def test_moved_operator_matches_oracle(name):
    wl = CASES[name]()
    print(f"[moving K] {wl.name}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=1, moving_body=1, amg_rebuild_every=2)
    P = Problem(wl, poisson_solver=0)
    err = _kdiff(ctx.poisson_matrix(), P.ops.K)
    print(f"  first positions: max entry difference {err:.2e}", flush=True)
    assert err < 1e-13
    h = wl.xf[len(wl.xf) // 2 + 1] - wl.xf[len(wl.xf) // 2]
    x = W.random_vector(ctx.n_lambda, 5)
    for k, (sx, sy) in enumerate(SHIFTS):
        xb, yb = wl.xb + sx * h, wl.yb + sy * h
        ub = (np.full(wl.nb, 0.1 * k), np.full(wl.nb, -0.2))
        ctx.move_body(xb, yb, *ub)
        P.move_body(xb, yb, *ub, hierarchy="keep")
        Kg = ctx.poisson_matrix()
        err = _kdiff(Kg, P.ops.K)
        ea = _rel(_n(ctx.apply_K(_t(x))), P.ops.K @ x)
        info = ctx.moving_info()
        print(f"  move {k + 1} ({sx:+.2f}, {sy:+.2f}) cells: nnz {Kg.nnz} vs {P.ops.K.nnz}; max entry "
              f"difference {err:.2e}; K x {ea:.2e}; box {info['box']}; refreshes {info['refreshes']}",
              flush=True)
        assert err < 1e-13 and ea < 1e-13
        assert info["moves"] == k + 1 and info["refreshes"] == (k + 1) // 2
        # K stays symmetric; the coupling blocks bit for bit (both sides of
        # the diagonal are the same sums in the same order)
        nc = ctx.n_lambda - 2 * wl.nb
        D = (Kg - Kg.T).tocoo()
        if D.nnz:
            a = int(np.argmax(np.abs(D.data)))
            print(f"    largest asymmetry {D.data[a]:.2e} at ({D.row[a]}, {D.col[a]}), n_cell {nc}", flush=True)
        Kc = Kg[:nc, nc:]
        Kf = Kg[nc:, :]
        sym_cf = abs(Kc - Kf[:, :nc].T).max()
        sym_ff = abs(Kf[:, nc:] - Kf[:, nc:].T).max()
        print(f"    coupling asymmetry {sym_cf:.2e}, force block {sym_ff:.2e}", flush=True)
        assert abs(Kg - Kg.T).max() <= 1e-15 * np.max(np.abs(Kg.data))
        assert sym_ff == 0.0
    ctx.close()


def test_moved_stages_match_oracle():
    """The Poisson right-hand side (E q* - u_B) and the projection
    (q* - B^1 (G phi + E^T f)) with the moved E."""
    wl = W.cylinder_small(96, 60)
    ctx = ibpm.Context(wl, poisson_solver=0, moving_body=1)
    P = Problem(wl, poisson_solver=0)
    h = wl.xf[1] - wl.xf[0]
    xb, yb = wl.xb + 0.41 * h, wl.yb - 0.73 * h
    ubx, uby = np.linspace(-0.3, 0.2, wl.nb), np.full(wl.nb, 0.15)
    ctx.move_body(xb, yb, ubx, uby)
    P.move_body(xb, yb, ubx, uby)
    rng = np.random.default_rng(11)
    qs = rng.standard_normal(ctx.n_q)
    lam = rng.standard_normal(ctx.n_lambda)
    walls = ctx.get_walls(1)
    st = P.initial_state()
    rhs = _n(ctx.stage_rhs2(_t(qs)))
    rhs_ref = flow.poisson_rhs(P.ops, qs, st.walls, P.ub)
    out = _n(ctx.stage_project(_t(qs), _t(lam)))
    ref = flow.project(P.ops, qs, lam)
    print(f"  rhs {_maxrel(rhs, rhs_ref):.2e} projection {_maxrel(out, ref):.2e}", flush=True)
    assert walls.size > 0
    assert _maxrel(rhs, rhs_ref) < 1e-12
    assert _maxrel(out, ref) < 1e-13
    ctx.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("solver,every", [(0, 0), (1, 0), (1, 1), (1, 3)])
def test_heaving_trajectory_matches_oracle(solver, every):
    """A cylinder heaving across the stream, moved before each step to its
    position at the time the step advances to."""
    wl = W.cylinder_small(96, 60).replace(poisson_solver=solver)
    print(f"[heave] solver {solver} refresh every {every}", flush=True)
    ctx = ibpm.Context(wl, poisson_solver=solver, moving_body=1, amg_rebuild_every=every,
                       vel_rtol=TIGHT, poisson_rtol=TIGHT, poisson_maxit=20000)
    P = Problem(wl, poisson_solver=solver, vel_rtol=TIGHT, poisson_rtol=TIGHT)
    P.wl = wl.replace(poisson_maxit=20000)
    q, conv, lam = ctx.init_state()
    st = P.initial_state()
    g_it, o_it = [], []
    for n in range(8):
        body = W.heave(wl, (n + 1) * wl.dt, amplitude=0.2, period=0.4)
        ctx.move_body(*body)
        P.move_body(*body, hierarchy="keep")
        s = ctx.step(q, conv, lam, 1)
        st, info = P.step(st)
        g_it.append(s["last_poisson_iters"])
        o_it.append(info.poisson_iters)
    R = P.grid.R_diag()
    eu = _rel(_n(q) / R, st.q / R)
    el = _rel(_n(lam), st.lam)
    print(f"  8 steps: velocity {eu:.2e} lambda {el:.2e}; Fy {s['fy']:.10f} vs {info.fy:.10f}; "
          f"iters {g_it} vs {o_it}", flush=True)
    assert eu < 1e-10 and el < 1e-10
    ctx.close()


def test_body_carried_by_the_stream_leaves_it_uniform():
    """A body moving with a uniform stream at the stream's velocity
    disturbs nothing: the flow stays uniform and the forces vanish."""
    wl = W.tiny(16, 14, 8, 0.2, stretched=False, dt=0.02, nu=0.05).replace(uinf=1.0, alpha=0.3)
    U, V = np.cos(0.3), np.sin(0.3)
    ctx = ibpm.Context(wl, poisson_solver=0, moving_body=1, vel_rtol=TIGHT, poisson_rtol=1e-13,
                       body_ramp=0.0)
    q, conv, lam = ctx.init_state()
    q0 = _n(q).copy()
    for n in range(6):
        t1 = (n + 1) * wl.dt
        ctx.move_body(wl.xb + U * t1, wl.yb + V * t1, np.full(wl.nb, U), np.full(wl.nb, V))
        ctx.step(q, conv, lam, 1)
    dq = np.max(np.abs(_n(q) - q0)) / np.max(np.abs(q0))
    f = np.max(np.abs(_n(lam)[ctx.n_lambda - 2 * wl.nb:]))
    print(f"  uniform stream after 6 moves: velocity change {dq:.2e}, largest force {f:.2e}", flush=True)
    assert dq < 1e-11 and f < 1e-10
    ctx.close()


def test_refreshed_hierarchy_matches_oracle_refresh():
    """The hierarchy formed anew on the device (aggregates and weights of
    the first set-up) against the oracle's refresh of the same hierarchy:
    the same level sizes, and AMG-PCG takes the same iterations on the
    moved K."""
    wl = W.cylinder_small(96, 60)
    ctx = ibpm.Context(wl, poisson_solver=1, moving_body=1, amg_rebuild_every=1)
    P = Problem(wl, poisson_solver=1)
    sizes0, _ = ctx.hierarchy()
    assert sizes0 == P.H.sizes()
    h = wl.xf[1] - wl.xf[0]
    b = W.random_vector(ctx.n_lambda, 21)
    b[wl.pin_cell] = 0.0
    for k, (sx, sy) in enumerate(SHIFTS[:3]):
        xb, yb = wl.xb + sx * h, wl.yb + sy * h
        z = np.zeros(wl.nb)
        ctx.move_body(xb, yb, z, z)
        P.move_body(xb, yb, z, z, hierarchy="refresh")
        sizes, nnz = ctx.hierarchy()
        no = [lev.A.nnz for lev in P.H.levels]
        lam = ctx.zeros_lambda()
        st = ctx.solve_poisson(_t(b), lam)
        x, it, _ = P.solve_poisson(b, np.zeros_like(b), rtol=wl.poisson_rtol, maxit=2000)
        el = _rel(_n(lam), x)
        print(f"  move {k + 1}: level nnz {nnz} vs {no}; iters {st['iters']} vs {it}; "
              f"solution {el:.2e}", flush=True)
        assert sizes == P.H.sizes()
        # entries that cancel exactly are dropped by the oracle's products
        assert all(abs(a - o) <= 0.002 * o for a, o in zip(nnz, no))
        assert abs(st["iters"] - it) <= 1
        assert el < 50 * wl.poisson_rtol
    ctx.close()


def test_move_errors_leave_the_context_unchanged():
    wl = W.cylinder_small(96, 60)
    fixed = ibpm.Context(wl, poisson_solver=0)
    z = np.zeros(wl.nb)
    with pytest.raises(ibpm.IBPMError):
        fixed.move_body(wl.xb, wl.yb, z, z)
    fixed.close()
    ctx = ibpm.Context(wl, poisson_solver=1, moving_body=1, amg_rebuild_every=1)
    K0 = ctx.poisson_matrix()
    for xb, yb in [(wl.xb + 1.9, wl.yb),                       # supports leave the grid
                   (wl.xb, np.where(np.arange(wl.nb) == 3, np.nan, wl.yb))]:
        with pytest.raises(ibpm.IBPMError):
            ctx.move_body(xb, yb, z, z)
    info = ctx.moving_info()
    assert info["moves"] == 0 and info["refreshes"] == 0
    assert abs(ctx.poisson_matrix() - K0).max() == 0.0
    ctx.close()


@pytest.mark.timeout(900)
def test_moved_rows_at_2048_match_oracle_products():
    """On the 2048^2 grid (4.2M cells, 628 points) the rows of K that a move
    changes -- the force rows and the coupled cells' rows -- against the
    products E B^1 G and E B^1 E^T formed from the oracle's E, B^1 and G at
    the moved positions; the pressure rows stay G^T B^1 G."""
    wl = W.heaving_cylinder(2048)
    ctx = ibpm.Context(wl, poisson_solver=1, moving_body=1, amg_rebuild_every=1)
    body = W.heave(wl, 0.3)
    ctx.move_body(*body)
    Kg = ctx.poisson_matrix()
    info = ctx.moving_info()
    grid = Grid(wl.xf, wl.yf)
    _, E = delta.interpolation_matrices(grid, body[0], body[1])
    B1 = wl.dt / (grid.M_diag() / grid.R_diag())
    G = operators.gradient(grid)
    EB = (E @ sp.diags(B1)).tocsr()
    Kfc = (EB @ G).tocsr()
    Kff = (EB @ E.T).tocsr()
    nc = grid.n_cell
    Kfc = Kfc.tolil()
    Kfc[:, wl.pin_cell] = 0.0
    Kfc = Kfc.tocsr()
    F = Kg[nc:, :]
    scale = abs(Kff).max()
    e_fc = abs(F[:, :nc] - Kfc).max() / scale
    e_ff = abs(F[:, nc:] - Kff).max() / scale
    # the coupled cells' rows: the transpose of the force rows
    e_cf = abs(Kg[:nc, nc:] - Kfc.T).max() / scale
    # pressure rows unchanged (against those of the first positions)
    Kp = (G.T @ sp.diags(B1) @ G).tocsr()
    Kp = operators.pin_matrix(Kp, wl.pin_cell)
    i0, i1, j0, j1 = info["box"]
    e_pp = abs(Kg[:nc, :nc] - Kp).max() / abs(Kp).max()
    print(f"  2048^2 moved K: {Kg.nnz} entries, box {info['box']}; force-cell {e_fc:.2e} force-force "
          f"{e_ff:.2e} cell-force {e_cf:.2e} pressure {e_pp:.2e}", flush=True)
    assert e_fc < 1e-13 and e_ff < 1e-13 and e_cf < 1e-13 and e_pp < 1e-13
    # the body's cells (a diameter of 200 cells) and two more on each side
    assert i1 - i0 < 220 and j1 - j0 < 220
    # a Poisson solve on the moved K with the hierarchy formed on the device
    b = W.random_vector(ctx.n_lambda, 2)
    b[wl.pin_cell] = 0.0
    lam = ctx.zeros_lambda()
    st = ctx.solve_poisson(_t(b), lam)
    print(f"  AMG-PCG on the moved K: {st['iters']} iterations, relres {st['relres']:.2e}", flush=True)
    assert st["status"] == 0 and st["relres"] <= wl.poisson_rtol
    ctx.close()
