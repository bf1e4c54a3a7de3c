"""How well the 512^2 Poisson solution lambda is determined by the data, in
the oracle (CPU): the basis for comparing lambda between two correct
solvers.

K = Q^T B^1 Q is ill-conditioned (its smallest eigenvalue belongs to the
interior-pressure / normal-force mode), so two exact solvers can differ in
lambda for two reasons:
  * rounding of K's entries: every stored entry multiplied by 1 + e with
    |e| <= 2^-53 (a last-bit difference in assembly) moves lambda by about
    1e-12 relative -- two orders below the 1e-10 bar;
  * the stopping point of the iteration: AMG-PCG stopped at a 1e-13
    relative residual differs from the direct (sparse LU) solution by about
    2e-12 (at 1e-8: 6e-9).
Velocity, the quantity the projection produces, moves by rounding only.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import flow, solvers
from oracle.problem import Problem
from paper_1109_3524_amd import workloads as W


@pytest.fixture(scope="module")
def first_step_512():
    wl = W.cylinder_512()
    P = Problem(wl)
    o, g = P.ops, P.grid
    st = P.initial_state()
    w1 = flow.update_walls(g, st.walls, st.q, wl.uinf, wl.alpha, o.dt)
    conv = flow.convection(g, st.q, st.walls)
    r1 = flow.momentum_rhs(o, st.q, conv, conv, st.walls, w1)
    qs = spla.spsolve(o.A.tocsc(), r1)
    rhs = flow.poisson_rhs(o, qs, w1, P.ub)
    lam = spla.spsolve(o.K.tocsc(), rhs)
    return P, qs, rhs, lam


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_last_bit_changes_of_K_move_lambda_far_below_1e10(first_step_512):
    P, qs, rhs, lam = first_step_512
    o = P.ops
    U = sp.triu(o.K, k=0).tocoo()
    rng = np.random.default_rng(1)
    for _ in range(2):
        eps = rng.uniform(-1.0, 1.0, U.nnz) * 2.0 ** -53
        Up = sp.csr_matrix((U.data * (1.0 + eps), (U.row, U.col)), shape=U.shape)
        Kp = (Up + sp.triu(Up, k=1).T).tocsc()
        lp = spla.spsolve(Kp, rhs)
        d_lam = _rel(lp, lam)
        d_q = _rel(qs - o.B1 * (o.Q @ lp), qs - o.B1 * (o.Q @ lam))
        assert 1e-14 < d_lam < 1e-11, d_lam
        assert d_q < 1e-13, d_q


def test_amg_pcg_stopping_error_at_1e13(first_step_512):
    P, qs, rhs, lam = first_step_512
    x, it, res = solvers.amg_pcg(P.H, P.ops.K, rhs, np.zeros_like(rhs), 1e-13, 5000)
    assert res < 2e-13
    assert _rel(x, lam) < 2e-11
