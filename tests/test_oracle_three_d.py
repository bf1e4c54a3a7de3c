"""Pins of the oracle's three-dimensional operators and time-step linear
algebra (the 7-point extension the paper names as its next step, Sec. 7;
Eqs. 6-11 carried over axis by axis).

- without a body and on a uniform grid the pressure block of K is dt h times
  the 7-point Neumann Laplacian built here from one-dimensional ones;
- E reproduces linear velocity fields exactly (the product of three deltas
  keeps each direction's moment conditions);
- A is symmetric positive definite; K is symmetric with rank n - 1 before
  the pressure value is pinned and positive definite after;
- one step's linear algebra leaves Q^T q = r2 (continuity and no-slip) and
  misses the momentum row by exactly (nu dt / 2) L Mf^-1 Q lambda, the
  defect of B^1 = dt Mf^-1 as an inverse of A (Eq. 11 against Eq. 10);
- with B = A^-1 the same three steps solve the saddle-point system of
  Eq. 10 itself."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import solvers, three_d as T3
from paper_1109_3524_amd import workloads as W


def _lap1(n):
    """1-D Neumann graph Laplacian (n nodes)."""
    main = np.full(n, 2.0)
    main[0] = main[-1] = 1.0
    return sp.diags([-np.ones(n - 1), main, -np.ones(n - 1)], [-1, 0, 1], format="csr")


def test_pressure_block_without_body_is_7_point_neumann_laplacian():
    nx, ny, nz = 6, 5, 4
    h = 0.25
    g = T3.Grid3(np.arange(nx + 1) * h, np.arange(ny + 1) * h, np.arange(nz + 1) * h)
    E = sp.csr_matrix((0, g.n_q))
    ops = T3.Operators3(g, E, nu=0.1, dt=0.02)
    Ix, Iy, Iz = (sp.identity(n) for n in (nx, ny, nz))
    L7 = (sp.kron(Iz, sp.kron(Iy, _lap1(nx))) + sp.kron(Iz, sp.kron(_lap1(ny), Ix)) +
          sp.kron(_lap1(nz), sp.kron(Iy, Ix)))
    ref = 0.02 * h * L7
    assert abs(ops.K_unpinned - ref).max() < 1e-15


def test_interpolation_reproduces_linear_fields():
    wl = W.sphere3d(12, n_b=30, radius=0.3)
    g = T3.Grid3(wl.xf, wl.yf, wl.zf)
    E = T3.interpolation_matrix(g, wl.xb, wl.yb, wl.zb)
    rng = np.random.default_rng(3)
    R = g.R_diag()
    for a in range(3):
        c = rng.standard_normal(4)
        pos = [g.f[b][1:-1] if b == a else g.c[b] for b in range(3)]
        Z, Y, X = np.meshgrid(pos[2], pos[1], pos[0], indexing="ij")
        u = c[0] + c[1] * X + c[2] * Y + c[3] * Z
        q = np.zeros(g.n_q)
        q[g.off[a]:g.off[a] + g.n_comp[a]] = u.ravel() * R[g.off[a]:g.off[a] + g.n_comp[a]]
        got = (E @ q)[a * wl.nb:(a + 1) * wl.nb]
        want = c[0] + c[1] * wl.xb + c[2] * wl.yb + c[3] * wl.zb
        assert np.max(np.abs(got - want)) < 1e-13 * max(1.0, np.max(np.abs(want)))
        # the other components' rows see nothing of this one
        other = np.delete(E @ q, np.arange(a * wl.nb, (a + 1) * wl.nb))
        assert np.max(np.abs(other)) == 0.0


@pytest.mark.parametrize("stretched", [False, True])
def test_A_spd_K_symmetric_rank_and_definiteness(stretched):
    wl = W.sphere3d(8, n_b=6, radius=0.15, stretched=stretched)
    g = T3.Grid3(wl.xf, wl.yf, wl.zf)
    ops = T3.Operators3(g, T3.interpolation_matrix(g, wl.xb, wl.yb, wl.zb), wl.nu, wl.dt)
    A = ops.A.toarray()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-12 * abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0
    Ku = ops.K_unpinned.toarray()
    np.testing.assert_allclose(Ku, Ku.T, rtol=0, atol=1e-14 * abs(Ku).max())
    s = np.linalg.svd(Ku, compute_uv=False)
    assert s[-1] < 1e-12 * s[0] and s[-2] > 1e-9 * s[0]
    Kp = ops.K.toarray()
    assert np.linalg.eigvalsh(Kp).min() > 0


def _rhs(ops, seed):
    rng = np.random.default_rng(seed)
    r1 = rng.standard_normal(ops.n_q)
    r2 = rng.standard_normal(ops.n_lambda)
    # the continuity rows must be consistent with a closed box: zero net flux
    nc = ops.grid.n_cell
    r2[:nc] -= r2[:nc].mean()
    return r1, r2


def test_linear_step_continuity_and_the_defect_of_b1():
    wl = W.sphere3d(10, n_b=20, radius=0.25)
    g = T3.Grid3(wl.xf, wl.yf, wl.zf)
    ops = T3.Operators3(g, T3.interpolation_matrix(g, wl.xb, wl.yb, wl.zb), wl.nu, wl.dt)
    r1, r2 = _rhs(ops, 4)
    q, lam, qs = T3.linear_step(ops, r1, r2, np.zeros(ops.n_q), np.zeros(ops.n_lambda), 1e-14, 1e-14)
    cont = ops.Q.T @ q - r2
    cont[ops.pin] = 0.0
    assert np.linalg.norm(cont) < 1e-10 * np.linalg.norm(r2)
    defect = ops.A @ q + ops.Q @ lam - r1
    expect = 0.5 * ops.nu * ops.dt * (ops.L @ ((ops.Q @ lam) / ops.Mf))
    assert np.linalg.norm(defect - expect) < 1e-10 * np.linalg.norm(expect)


def test_exact_factorisation_solves_the_saddle_point_system():
    """With B = A^-1 the three steps give the solution of Eq. 10."""
    wl = W.sphere3d(6, n_b=4, radius=0.2)
    g = T3.Grid3(wl.xf, wl.yf, wl.zf)
    ops = T3.Operators3(g, T3.interpolation_matrix(g, wl.xb, wl.yb, wl.zb), wl.nu, wl.dt)
    r1, r2 = _rhs(ops, 5)
    A = ops.A.toarray()
    Q = ops.Q.toarray()
    Ainv = np.linalg.inv(A)
    qs = Ainv @ r1
    K = Q.T @ Ainv @ Q
    p = ops.pin
    keep = np.arange(ops.n_lambda) != p
    lam = np.zeros(ops.n_lambda)
    lam[keep] = np.linalg.solve(K[np.ix_(keep, keep)], (Q.T @ qs - r2)[keep])
    q = qs - Ainv @ (Q @ lam)
    assert np.linalg.norm(A @ q + Q @ lam - r1) < 1e-10 * np.linalg.norm(r1)
    res = Q.T @ q - r2
    assert np.linalg.norm(res[keep]) < 1e-10 * np.linalg.norm(r2)
    # the dense saddle-point solve (pinned unknown removed) gives the same
    n = ops.n_q
    S = np.block([[A, Q[:, keep]], [Q[:, keep].T, np.zeros((keep.sum(), keep.sum()))]])
    sol = np.linalg.solve(S, np.concatenate([r1, r2[keep]]))
    assert np.linalg.norm(sol[:n] - q) < 1e-9 * np.linalg.norm(q)
    assert np.linalg.norm(sol[n:] - lam[keep]) < 1e-9 * np.linalg.norm(lam)


def test_amg_and_jacobi_pcg_agree_on_the_3d_system():
    wl = W.sphere3d(12, n_b=30, radius=0.3)
    g = T3.Grid3(wl.xf, wl.yf, wl.zf)
    ops = T3.Operators3(g, T3.interpolation_matrix(g, wl.xb, wl.yb, wl.zb), wl.nu, wl.dt)
    rng = np.random.default_rng(6)
    b = rng.standard_normal(ops.n_lambda)
    b[ops.pin] = 0.0
    H = solvers.SAHierarchy(ops.K, coarse_max=64)
    assert len(H.levels) >= 2
    x1, _, _ = solvers.amg_pcg(H, ops.K, b, np.zeros_like(b), 1e-13, 5000)
    x2, _, _ = solvers.jacobi_pcg(ops.K, b, np.zeros_like(b), 1e-13, 20000)
    assert np.linalg.norm(x1 - x2) < 1e-9 * np.linalg.norm(x2)
