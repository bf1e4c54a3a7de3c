"""Pins of the oracle's assembled operators against what the discrete
formulation fixes: consistency with the continuous operators (order of
accuracy), symmetry and definiteness (Sec. 2, last paragraph), the null
space of Q^T B Q before pinning, the classical projection-method pressure
operator in the absence of a body, and the unknown counts of Sec. 3,
Table "test_details"."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import delta, flow, operators
from oracle.grid import Grid
from paper_1109_3524_amd import workloads as W


def _ops(wl):
    g = Grid(wl.xf, wl.yf)
    Eh, E = delta.interpolation_matrices(g, wl.xb, wl.yb)
    return operators.Operators(g, E, wl.nu, wl.dt)


def _walls_from(g, fu, fv):
    """Wall values sampled from exact functions at the wall positions."""
    w = flow.freestream_walls(g, 0.0, 0.0)
    w.uL = fu(g.xf[0], g.yc)
    w.uR = fu(g.xf[-1], g.yc)
    w.vB = fv(g.xc, g.yf[0])
    w.vT = fv(g.xc, g.yf[-1])
    w.uBt = fu(g.xf, g.yf[0])
    w.uTt = fu(g.xf, g.yf[-1])
    w.vLt = fv(g.xf[0], g.yf)
    w.vRt = fv(g.xf[-1], g.yf)
    return w


def _sample_q(g, fu, fv):
    xu, yu = np.meshgrid(g.xf[1:-1], g.yc)
    xv, yv = np.meshgrid(g.xc, g.yf[1:-1])
    return g.join_q(fu(xu, yu), fv(xv, yv)) * g.R_diag()


fu = lambda x, y: np.sin(1.3 * x + 0.4) * np.cos(0.9 * y - 0.2) + 0.5
fv = lambda x, y: np.cos(0.7 * x - 0.3) * np.sin(1.1 * y + 0.1) - 0.25


def _lap_exact(x, y, which):
    if which == "u":
        return -(1.3 ** 2 + 0.9 ** 2) * np.sin(1.3 * x + 0.4) * np.cos(0.9 * y - 0.2)
    return -(0.7 ** 2 + 1.1 ** 2) * np.cos(0.7 * x - 0.3) * np.sin(1.1 * y + 0.1)


def _conv_exact(x, y, which):
    # d(uu)/dx + d(uv)/dy for u-momentum; d(uv)/dx + d(vv)/dy for v-momentum
    u = fu(x, y)
    v = fv(x, y)
    ux = 1.3 * np.cos(1.3 * x + 0.4) * np.cos(0.9 * y - 0.2)
    uy = -0.9 * np.sin(1.3 * x + 0.4) * np.sin(0.9 * y - 0.2)
    vx = -0.7 * np.sin(0.7 * x - 0.3) * np.sin(1.1 * y + 0.1)
    vy = 1.1 * np.cos(0.7 * x - 0.3) * np.cos(1.1 * y + 0.1)
    if which == "u":
        return 2 * u * ux + uy * v + u * vy
    return ux * v + u * vx + 2 * v * vy


def _interior_err(g, vec_scaled, which_fn):
    """max error of (vec / M) against the exact operator, two unknowns away
    from every wall."""
    M = g.M_diag()
    r = vec_scaled / M
    ru, rv = g.split_q(r)
    xu, yu = np.meshgrid(g.xf[1:-1], g.yc)
    xv, yv = np.meshgrid(g.xc, g.yf[1:-1])
    eu = np.abs(ru - which_fn(xu, yu, "u"))[2:-2, 2:-2]
    ev = np.abs(rv - which_fn(xv, yv, "v"))[2:-2, 2:-2]
    return max(eu.max(), ev.max())


def _order(errs):
    return [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_laplacian_matrix_matches_explicit_differences():
    wl = W.tiny(14, 12, 0, stretched=True)
    o = _ops(wl)
    g = o.grid
    q = np.random.default_rng(1).standard_normal(g.n_q)
    walls = flow.freestream_walls(g, 1.0, 0.2)
    walls.uR = walls.uR + np.linspace(0, 0.3, g.ny)
    walls.vRt = walls.vRt + np.linspace(0, -0.2, g.ny + 1)
    a = flow.laplacian_full(g, q, walls)
    b = o.L @ q + o.Md * operators.laplacian_bc(g, walls)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("stretched", [False, True])
def test_laplacian_converges_to_continuous(stretched):
    errs = []
    for n in (16, 32, 64):
        if stretched:
            xf = W.stretched_faces(n, 1.5, 0.5, 1.0 / (n // 2))
        else:
            xf = W.uniform_faces(n, -1.0, 1.0)
        g = Grid(xf, xf)
        walls = _walls_from(g, fu, fv)
        lap = flow.laplacian_full(g, _sample_q(g, fu, fv), walls)
        errs.append(_interior_err(g, lap, _lap_exact))
    orders = _order(errs)
    assert min(orders) > (1.8 if not stretched else 0.9), (errs, orders)


def test_convection_converges_to_continuous():
    errs = []
    for n in (16, 32, 64, 128):
        xf = W.uniform_faces(n, -1.0, 1.0)
        g = Grid(xf, xf)
        walls = _walls_from(g, fu, fv)
        N = flow.convection(g, _sample_q(g, fu, fv), walls)
        errs.append(_interior_err(g, N, _conv_exact))
    orders = _order(errs)
    assert min(orders[1:]) > 1.8, (errs, orders)


def test_convection_of_uniform_flow_vanishes():
    wl = W.tiny(14, 12, 0, stretched=True)
    g = Grid(wl.xf, wl.yf)
    walls = flow.freestream_walls(g, 1.0, 0.3)
    q = flow.freestream_flux(g, 1.0, 0.3)
    assert np.abs(flow.convection(g, q, walls)).max() < 1e-14


def test_divergence_gradient_relation_and_linear_flux():
    wl = W.tiny(12, 10, 0)
    o = _ops(wl)
    assert (o.G + o.D.T).nnz == 0 or np.abs((o.G + o.D.T).data).max() == 0.0
    g = o.grid
    # a uniform flow has zero full divergence in every cell
    q = flow.freestream_flux(g, 1.0, 0.7)
    walls = flow.freestream_walls(g, 1.0, 0.7)
    div = o.D @ q + flow.wall_flux_divergence(g, walls)
    assert np.abs(div).max() < 1e-15


@pytest.mark.parametrize("stretched", [False, True])
def test_K_symmetric_nullspace_rank_and_definiteness(stretched):
    wl = W.tiny(14, 12, 6, 0.2, stretched=stretched)
    o = _ops(wl)
    K = o.K_unpinned.toarray()
    n = K.shape[0]
    assert n == o.grid.n_cell + 2 * wl.nb
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-15 * np.abs(K).max())
    ones = np.concatenate([np.ones(o.grid.n_cell), np.zeros(2 * wl.nb)])
    assert np.abs(K @ ones).max() < 1e-14 * np.abs(K).max()
    s = np.linalg.svd(K, compute_uv=False)
    assert s[-1] < 1e-13 * s[0]          # one zero singular value ...
    assert s[-2] > 1e-8 * s[0]           # ... and only one
    Kp = o.K.toarray()
    np.linalg.cholesky(Kp)               # SPD after pinning
    np.linalg.cholesky(o.A.toarray())    # velocity operator SPD
    A = o.A.toarray()
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-15 * np.abs(A).max())


def test_pressure_block_is_classical_neumann_laplacian():
    # uniform square cells, no body: Q^T B Q = dt * (5-point Neumann Laplacian)
    n = 8
    xf = W.uniform_faces(n, 0.0, 1.0)
    g = Grid(xf, xf)
    E = sp.csr_matrix((0, g.n_q))
    dt = 0.37
    o = operators.Operators(g, E, 0.01, dt)
    K = o.K_unpinned.toarray()
    ref = np.zeros((n * n, n * n))
    for j in range(n):
        for i in range(n):
            c = j * n + i
            for (di, dj) in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    ref[c, c] += dt
                    ref[c, jj * n + ii] -= dt
    np.testing.assert_allclose(K, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("stretched", [False, True])
def test_manufactured_pressure_poisson_converges(stretched):
    errs = []
    for n in (16, 32, 64):
        if stretched:
            xf = W.stretched_faces(n, 1.5, 0.5, 1.0 / (n // 2))
        else:
            xf = W.uniform_faces(n, -1.0, 1.0)
        g = Grid(xf, xf)
        lo, hi = xf[0], xf[-1]
        L = hi - lo
        E = sp.csr_matrix((0, g.n_q))
        o = operators.Operators(g, E, 0.01, 1.0)
        X, Y = np.meshgrid(g.xc, g.yc)
        k = np.pi / L
        phi = np.cos(k * (X - lo)) * np.cos(k * (Y - lo))
        area = np.outer(g.dy, g.dx)
        rhs = (area * 2 * k * k * phi).ravel()
        rhs -= rhs.mean()                   # exact compatibility
        sol = sla.lstsq(o.K_unpinned.toarray(), rhs)[0]
        e = (sol - sol.mean()) - (phi.ravel() - phi.mean())
        errs.append(np.abs(e).max())
    orders = _order(errs)
    assert min(orders) > (1.8 if not stretched else 1.5), (errs, orders)


def test_unknown_counts_of_the_solver_study(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "test_details_table.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 4
    for r in rows:
        nx, ny, nb, unknowns = int(r[1]), int(r[2]), int(r[3]), int(r[4])
        g = Grid(W.uniform_faces(nx, 0.0, 1.0), W.uniform_faces(ny, 0.0, 1.0))
        assert g.n_cell + 2 * nb == unknowns
    # and the assembled operator has exactly that many rows
    wl = W.cylinder_small(48, 30)
    o = _ops(wl)
    assert o.K.shape == (48 * 48 + 2 * 30,) * 2
