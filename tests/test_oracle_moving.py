"""Pins of the oracle's moving-body step (Sec. 6): the Lagrangian points
move between steps, and each step uses E and K at the new positions.

Special case: a body carried by a uniform stream at the stream's own
velocity disturbs nothing, so the flow stays uniform and the boundary
forces vanish, whatever the positions -- a step that kept the old E, or
took the old velocity, would disturb the flow."""
import numpy as np

from oracle.problem import Problem
from paper_1109_3524_amd import workloads as W


def test_body_carried_by_the_stream_leaves_it_uniform():
    wl = W.tiny(16, 14, 8, 0.2, stretched=False, dt=0.02, nu=0.05).replace(uinf=1.0, alpha=0.3)
    U, V = np.cos(0.3), np.sin(0.3)
    P = Problem(wl, vel_rtol=1e-13, poisson_rtol=1e-13)
    st = P.initial_state()
    q0 = st.q.copy()
    for n in range(6):
        t1 = (n + 1) * wl.dt
        xb, yb = wl.xb + U * t1, wl.yb + V * t1
        P.move_body(xb, yb, np.full(wl.nb, U), np.full(wl.nb, V))
        st, info = P.step(st)
    assert np.max(np.abs(st.q - q0)) < 1e-11 * np.max(np.abs(q0))
    assert np.max(np.abs(st.lam[P.grid.n_cell:])) < 1e-10


def test_moving_body_is_not_the_fixed_one():
    """The same points moved by half a cell give another solution than the
    fixed body (the step does use the new E)."""
    wl = W.tiny(16, 14, 8, 0.2, dt=0.02, nu=0.05)
    P1 = Problem(wl, vel_rtol=1e-13, poisson_rtol=1e-13)
    P2 = Problem(wl, vel_rtol=1e-13, poisson_rtol=1e-13)
    h = wl.xf[1] - wl.xf[0]
    P2.move_body(wl.xb + 0.5 * h, wl.yb, np.zeros(wl.nb), np.zeros(wl.nb))
    s1, _ = P1.step(P1.initial_state())
    s2, _ = P2.step(P2.initial_state())
    assert np.linalg.norm(s1.q - s2.q) > 1e-3 * np.linalg.norm(s1.q)


def test_refresh_on_the_same_operator_is_the_first_setup():
    """Forming the hierarchy anew on its own aggregates and weights from the
    operator it was set up on gives that set-up back (the refresh adds no
    step of its own), and on a moved K its coarse operators stay
    symmetric positive definite Galerkin products."""
    from oracle import solvers
    wl = W.tiny(24, 22, 12, 0.2, dt=0.02, nu=0.05)
    P = Problem(wl, poisson_solver=1)
    H = P.H
    assert len(H.levels) >= 2
    ref = [(lev.A.copy(), None if lev.P is None else lev.P.copy()) for lev in H.levels]
    H.refresh(P.ops.K)
    for (A0, P0), lev in zip(ref, H.levels):
        assert abs(A0 - lev.A).max() == 0.0
        if P0 is not None:
            assert abs(P0 - lev.P).max() == 0.0
    h = wl.xf[1] - wl.xf[0]
    P.move_body(wl.xb + 0.3 * h, wl.yb - 0.2 * h, np.zeros(wl.nb), np.zeros(wl.nb), hierarchy="refresh")
    for l, lev in enumerate(P.H.levels[1:]):
        A = lev.A.toarray()
        assert np.allclose(A, A.T, rtol=0, atol=1e-12 * abs(A).max())
        assert np.linalg.eigvalsh(A).min() > 0
    # a preconditioner built for another K still leaves the solution of
    # this K's system to the Krylov solve
    rng = np.random.default_rng(3)
    b = rng.standard_normal(P.ops.K.shape[0])
    b[wl.pin_cell] = 0.0
    for mode in ("keep", "refresh", "new"):
        P.move_body(wl.xb + 0.6 * h, wl.yb, np.zeros(wl.nb), np.zeros(wl.nb), hierarchy=mode)
        x, it, _ = P.solve_poisson(b, np.zeros_like(b), rtol=1e-12, maxit=400)
        assert np.linalg.norm(b - P.ops.K @ x) <= 1.01e-12 * np.linalg.norm(b)
