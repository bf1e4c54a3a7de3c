"""Pins of the oracle's B^N (Sec. 2, text after Eq. 11): the N-term
truncation of the Neumann series of A^{-1}, and the Poisson operator
K = Q^T B^N Q built from it.

With T = (nu dt / 2) L Mf^{-1}, A = Mf/dt - (nu/2) L = (I - T) Mf/dt and
B^N = dt Mf^{-1} sum_{k<N} T^k, so A B^N = I - T^N exactly (the sum
telescopes): the defect of B^N as an inverse of A is T^N, of order
(nu dt / h^2)^N."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import delta, operators
from oracle.grid import Grid
from paper_1109_3524_amd import workloads as W


def _ops(wl, n):
    g = Grid(wl.xf, wl.yf)
    _, E = delta.interpolation_matrices(g, wl.xb, wl.yb)
    return operators.Operators(g, E, wl.nu, wl.dt, bn_order=n)


@pytest.mark.parametrize("wl", [W.tiny(12, 10, 6), W.tiny(14, 12, 6, radius=0.2, stretched=True)],
                         ids=["uniform", "stretched"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_a_times_bn_is_identity_minus_t_to_the_n(wl, n):
    o = _ops(wl, n)
    T = (0.5 * o.nu * o.dt * o.L @ sp.diags(1.0 / o.Mf)).toarray()
    lhs = (o.A @ o.B).toarray()
    rhs = np.eye(o.n_q) - np.linalg.matrix_power(T, n)
    assert np.max(np.abs(lhs - rhs)) < 1e-13 * max(1.0, np.max(np.abs(lhs)))


@pytest.mark.parametrize("n", [1, 2, 3])
def test_bn_and_kn_are_symmetric_and_kn_spd(n):
    wl = W.tiny(12, 10, 6)
    o = _ops(wl, n)
    B = o.B.toarray()
    assert np.max(np.abs(B - B.T)) <= 1e-15 * np.max(np.abs(B))
    K = o.K.toarray()
    assert np.max(np.abs(K - K.T)) <= 1e-14 * np.max(np.abs(K))
    assert np.linalg.eigvalsh(0.5 * (K + K.T)).min() > 0


def test_bn_converges_to_the_inverse_of_a():
    """The defect |(B^N - A^{-1}) x| falls by about the spectral radius of T
    per added term."""
    wl = W.tiny(12, 10, 6).replace(dt=0.05, nu=0.05)
    x = W.random_vector(_ops(wl, 1).n_q, 3)
    Ainv_x = np.linalg.solve(_ops(wl, 1).A.toarray(), x)
    errs = [np.linalg.norm(_ops(wl, n).B @ x - Ainv_x) for n in (1, 2, 3, 4)]
    o = _ops(wl, 1)
    T = (0.5 * o.nu * o.dt * o.L @ sp.diags(1.0 / o.Mf)).toarray()
    rho = np.max(np.abs(np.linalg.eigvals(T)))
    assert rho < 1.0
    for a, b in zip(errs, errs[1:]):
        assert b < 1.05 * rho * a


def test_kn_widens_the_pressure_stencil():
    """Without a body, row (i, j) of the pressure block of Q^T B^N Q reaches
    the cells within Manhattan distance N of (i, j) (G and G^T add one cell
    each, every L one more)."""
    wl = W.tiny(16, 14, 0)
    for n in (1, 2, 3):
        o = _ops(wl, n)
        K = o.K_unpinned.tocsr()
        nx = wl.nx
        c = 7 * nx + 8
        cols = K.indices[K.indptr[c]:K.indptr[c + 1]]
        d = np.abs(cols % nx - 8) + np.abs(cols // nx - 7)
        assert d.max() == n
        assert len(cols) == 2 * n * n + 2 * n + 1
