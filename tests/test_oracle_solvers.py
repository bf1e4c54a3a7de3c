"""Pins of the oracle's solvers: brute-force dense solves on tiny grids,
hand-worked aggregation examples, and the structural properties a
smoothed-aggregation V-cycle preconditioner must have (symmetric, positive
definite) for PCG to be valid (Sec. 3)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import delta, operators, solvers
from oracle.grid import Grid
from paper_1109_3524_amd import workloads as W


def _ops(wl):
    g = Grid(wl.xf, wl.yf)
    Eh, E = delta.interpolation_matrices(g, wl.xb, wl.yb)
    return operators.Operators(g, E, wl.nu, wl.dt)


def _graph(name):
    if name == "chain7":
        n, edges = 7, [(i, i + 1) for i in range(6)]
    elif name == "chain4":
        n, edges = 4, [(0, 1), (1, 2), (2, 3)]
    elif name == "grid3x3":
        n = 9
        edges = []
        for r in range(3):
            for c in range(3):
                if c < 2:
                    edges.append((3 * r + c, 3 * r + c + 1))
                if r < 2:
                    edges.append((3 * r + c, 3 * r + c + 3))
    elif name == "star5":
        n, edges = 5, [(0, 1), (0, 2), (0, 3)]
    rows = [a for a, b in edges] + [b for a, b in edges]
    cols = [b for a, b in edges] + [a for a, b in edges]
    S = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    S.sort_indices()
    return S


def test_aggregation_hand_examples(golden_dir):
    for line in open(os.path.join(golden_dir, "aggregation_examples.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        parts = line.split()
        expect = np.array([int(x) for x in parts[1:]])
        agg, nagg = solvers.aggregate(_graph(parts[0]))
        np.testing.assert_array_equal(agg, expect, err_msg=parts[0])
        assert nagg == expect.max() + 1


def test_strength_drops_roundoff_residue():
    A = sp.csr_matrix(np.array([[2.0, -1.0, 1e-20], [-1.0, 2.0, -1.0], [1e-20, -1.0, 2.0]]))
    S = solvers.strength(A, 0.0).toarray()
    assert S[0, 2] == 0 and S[2, 0] == 0
    assert S[0, 1] == 1 and S[1, 2] == 1
    assert np.all(np.diag(S) == 0)


def test_gershgorin_bounds_spectral_radius():
    o = _ops(W.tiny(12, 10, 6))
    K = o.K.toarray()
    d = np.diag(K)
    rho = np.abs(np.linalg.eigvals(K / d[:, None])).max()
    assert solvers.gershgorin_rho(o.K) >= rho - 1e-12


@pytest.mark.parametrize("stretched", [False, True])
def test_pcg_matches_dense_solve(stretched):
    wl = W.tiny(14, 12, 6, 0.2, stretched=stretched)
    o = _ops(wl)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(o.K.shape[0])
    b[0] = 0.0
    exact = np.linalg.solve(o.K.toarray(), b)
    x, it, res = solvers.jacobi_pcg(o.K, b, np.zeros_like(b), 1e-14, 5000)
    assert np.linalg.norm(x - exact) <= 1e-12 * np.linalg.norm(exact)
    H = solvers.SAHierarchy(o.K, coarse_max=16)
    assert len(H.levels) >= 2
    x2, it2, res2 = solvers.amg_pcg(H, o.K, b, np.zeros_like(b), 1e-14, 5000)
    assert np.linalg.norm(x2 - exact) <= 1e-12 * np.linalg.norm(exact)
    bq = rng.standard_normal(o.A.shape[0])
    xq, _, _ = solvers.jacobi_pcg(o.A, bq, np.zeros_like(bq), 1e-14, 5000)
    exact_q = np.linalg.solve(o.A.toarray(), bq)
    assert np.linalg.norm(xq - exact_q) <= 1e-12 * np.linalg.norm(exact_q)


def test_vcycle_is_symmetric_positive_definite():
    wl = W.tiny(16, 14, 6, 0.2)
    o = _ops(wl)
    H = solvers.SAHierarchy(o.K, coarse_max=20)
    assert len(H.levels) >= 3
    n = o.K.shape[0]
    Minv = np.column_stack([H.vcycle(e) for e in np.eye(n)])
    np.testing.assert_allclose(Minv, Minv.T, rtol=0, atol=1e-10 * np.abs(Minv).max())
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0
    # Galerkin coarse operators are symmetric positive definite
    for lev in H.levels[1:]:
        Ac = lev.A.toarray()
        np.testing.assert_allclose(Ac, Ac.T, rtol=0, atol=1e-13 * np.abs(Ac).max())
        np.linalg.cholesky(Ac)


def test_aggregates_partition_and_constant_is_preserved():
    wl = W.cylinder_small(48, 30)
    o = _ops(wl)
    H = solvers.SAHierarchy(o.K)
    for lev in H.levels[:-1]:
        agg = lev.agg
        n = lev.A.shape[0]
        assert agg.min() == 0 and agg.max() == lev.P.shape[1] - 1
        assert len(np.unique(agg)) == lev.P.shape[1]
        # every aggregate is connected in the strength graph
        S = solvers.strength(lev.A, 0.0)
        for a in np.unique(agg)[:50]:
            members = np.nonzero(agg == a)[0]
            if len(members) == 1:
                continue
            sub = S[members][:, members]
            ncomp = sp.csgraph.connected_components(sub, directed=False)[0]
            assert ncomp == 1


def test_pcg_zero_rhs_and_immediate_convergence():
    o = _ops(W.tiny(12, 10, 4))
    b = np.zeros(o.K.shape[0])
    x, it, res = solvers.jacobi_pcg(o.K, b, np.ones_like(b), 1e-8, 100)
    assert it == 0 and np.all(x == 0)
    b = np.random.default_rng(0).standard_normal(o.K.shape[0])
    b[0] = 0
    exact = np.linalg.solve(o.K.toarray(), b)
    x, it, res = solvers.jacobi_pcg(o.K, b, exact, 1e-8, 100)
    assert it == 0


def test_splitmix64_start_vector_matches_published_outputs():
    # splitmix64 seeded with 0 (Steele, Lea & Flood 2014; the generator of
    # Java's SplittableRandom): the first two outputs are the published test
    # values 0xe220a8397b1dcdaf and 0x6e789e6aa1b965f4
    v = solvers.splitmix64_unit(2)
    for got, word in zip(v, (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4)):
        assert got == (word >> 11) / 2.0 ** 53 - 0.5
    w = solvers.splitmix64_unit(100000)
    assert -0.5 <= w.min() and w.max() < 0.5 and abs(w.mean()) < 0.005


@pytest.mark.parametrize("wl", [W.tiny(12, 10, 6), W.tiny(16, 14, 6, 0.2, stretched=True),
                                W.cylinder_small(96, 60)])
def test_lanczos_estimate_of_the_jacobi_spectral_radius(wl):
    # the Ritz estimate behind the SA weights lies within 1 % below the true
    # rho(D^-1 K) on every level (dense eigenvalues on the small levels,
    # ARPACK on the 96^2 finest level), so every damped-Jacobi smoother
    # w D^-1 with w = 4 / (3 rho_est) keeps w * rho_true < 2 (convergent)
    import scipy.sparse.linalg as sla
    o = _ops(wl)
    H = solvers.SAHierarchy(o.K, coarse_max=16)
    assert len(H.levels) >= 2
    for lev in H.levels:
        A = lev.A
        s = sp.diags(1.0 / np.sqrt(A.diagonal()))
        S = (s @ A @ s).tocsr()
        if A.shape[0] <= 2000:
            true = np.linalg.eigvalsh(S.toarray())[-1]
        else:
            true = sla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-12)[0]
        assert lev.rho <= true * (1 + 1e-12)
        assert lev.rho >= 0.99 * true, (A.shape[0], lev.rho, true)
        assert lev.omega * true < 2.0
        assert lev.rho < solvers.gershgorin_rho(A)


def test_lanczos_estimate_is_exact_on_a_known_spectrum():
    # D^-1 A for the 1-D Dirichlet Laplacian tridiag(-1, 2, -1) has the
    # eigenvalues 1 - cos(k pi / (n + 1)); with as many steps as unknowns
    # Lanczos reproduces the largest one to rounding
    n = 20
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    assert abs(solvers.lanczos_rho(A, steps=n) - (1 - np.cos(n * np.pi / (n + 1)))) < 1e-13
    # a diagonal matrix with a scaled diagonal: D^-1 A = I, rho = 1 exactly
    B = sp.diags(np.linspace(1.0, 5.0, 30), format="csr")
    assert abs(solvers.lanczos_rho(B) - 1.0) < 1e-14
