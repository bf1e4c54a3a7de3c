"""Assembled sparse operators of the transformed system (Sec. 2, Eqs. 8-11).

Oracle code: test infrastructure only.

The paper defers the symmetrising transformation to Taira & Colonius; the
reading used here makes every operator explicit:
  R   = diag(dy_j | dx_i)           q = R u (flux through each face)
  M   = diag(Dx_i | Dy_j)           row scaling of the momentum equations
  Mf  = M R^{-1}                    flux "mass" matrix
  D   interior-face divergence:     (Dq)_c = q^u_{i+1,j}-q^u_{i,j}+q^v_{i,j+1}-q^v_{i,j}
  G   = -D^T                        (G phi)^u_{i,j} = phi_{i,j} - phi_{i-1,j}
  L   = M Lhat R^{-1}               Lhat: 3-point second differences (non-uniform)
  A   = Mf/dt - (nu/2) L            Crank-Nicolson implicit operator (Sec. 2, text before Eq. 8)
  B^1 = dt Mf^{-1}                  first-order approximation of A^{-1} (Eq. 11, N = 1)
  B^N = dt Mf^{-1} sum_{k<N} ((nu dt/2) L Mf^{-1})^k
                                    N-term truncation of the Neumann series of
                                    A^{-1} = dt Mf^{-1} (I - (nu dt/2) L Mf^{-1})^{-1}
                                    (Sec. 2, text after Eq. 11; N = 3 in Sec. 5.1)
  Q   = [G, E^T]                    Eq. (9)
  K   = Q^T B^N Q                   left-hand side of Eq. (11b)
Wall values enter Lhat through boundary vectors (`laplacian_bc`): normal
velocities sit on the wall (a full cell away from the first unknown),
tangential ones sit on the wall half a cell from the first unknown.

One pressure value is pinned (Sec. 2, last paragraph): the reading is cell
(0,0), with row and column 0 cleared except the diagonal.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def divergence(grid):
    """D: (n_cell x n_q), interior faces only."""
    nx, ny = grid.nx, grid.ny
    rows, cols, vals = [], [], []
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    c = grid.cidx(I, J)
    # east face u_{i+1,j} (+1) if interior
    m = I + 1 <= nx - 1
    rows.append(c[m]); cols.append(grid.uidx(I[m] + 1, J[m])); vals.append(np.ones(m.sum()))
    # west face u_{i,j} (-1) if interior
    m = I >= 1
    rows.append(c[m]); cols.append(grid.uidx(I[m], J[m])); vals.append(-np.ones(m.sum()))
    # north face v_{i,j+1} (+1)
    m = J + 1 <= ny - 1
    rows.append(c[m]); cols.append(grid.vidx(I[m], J[m] + 1)); vals.append(np.ones(m.sum()))
    # south face v_{i,j} (-1)
    m = J >= 1
    rows.append(c[m]); cols.append(grid.vidx(I[m], J[m])); vals.append(-np.ones(m.sum()))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(grid.n_cell, grid.n_q))


def gradient(grid):
    """G = -D^T."""
    return (-divergence(grid).T).tocsr()


def _second_difference(centre_gap, left_gap, right_gap):
    """1-D 3-point second difference on n nodes.

    Row m: [ 1/left_gap[m], -(1/left_gap[m] + 1/right_gap[m]), 1/right_gap[m] ] / centre_gap[m],
    the outer entries of the first and last rows dropped (they multiply wall values).
    """
    n = len(centre_gap)
    lo = 1.0 / (left_gap * centre_gap)
    hi = 1.0 / (right_gap * centre_gap)
    main = -(lo + hi)
    return sp.diags([lo[1:], main, hi[:-1]], [-1, 0, 1], shape=(n, n), format="csr")


def laplacian_hat(grid):
    """Lhat on interior velocity unknowns (block diagonal u / v)."""
    nx, ny = grid.nx, grid.ny
    dx, dy, Dx, Dy = grid.dx, grid.dy, grid.Dx, grid.Dy
    # u: x-nodes x_1..x_{nx-1} (gaps dx), y-nodes yc_0..yc_{ny-1} (gaps Dy)
    Lx_u = _second_difference(Dx[1:-1], dx[:-1], dx[1:])
    Ly_u = _second_difference(dy, Dy[:-1], Dy[1:])
    Lu = sp.kron(sp.identity(ny), Lx_u) + sp.kron(Ly_u, sp.identity(nx - 1))
    # v: x-nodes xc_0..xc_{nx-1} (gaps Dx), y-nodes y_1..y_{ny-1} (gaps dy)
    Lx_v = _second_difference(dx, Dx[:-1], Dx[1:])
    Ly_v = _second_difference(Dy[1:-1], dy[:-1], dy[1:])
    Lv = sp.kron(sp.identity(ny - 1), Lx_v) + sp.kron(Ly_v, sp.identity(nx))
    return sp.block_diag([Lu, Lv], format="csr")


def laplacian_bc(grid, bc):
    """Contribution of wall values to Lhat u (velocity units, not row-scaled)."""
    nx, ny = grid.nx, grid.ny
    dx, dy, Dx, Dy = grid.dx, grid.dy, grid.Dx, grid.Dy
    bu = np.zeros((ny, nx - 1))
    bv = np.zeros((ny - 1, nx))
    # u rows: normal wall values left/right (gap dx), tangential bottom/top (gap Dy)
    bu[:, 0] += bc.uL / (dx[0] * Dx[1])
    bu[:, -1] += bc.uR / (dx[-1] * Dx[nx - 1])
    bu[0, :] += bc.uBt[1:nx] / (Dy[0] * dy[0])
    bu[-1, :] += bc.uTt[1:nx] / (Dy[ny] * dy[ny - 1])
    # v rows: normal wall values bottom/top (gap dy), tangential left/right (gap Dx)
    bv[0, :] += bc.vB / (dy[0] * Dy[1])
    bv[-1, :] += bc.vT / (dy[-1] * Dy[ny - 1])
    bv[:, 0] += bc.vLt[1:ny] / (Dx[0] * dx[0])
    bv[:, -1] += bc.vRt[1:ny] / (Dx[nx] * dx[nx - 1])
    return grid.join_q(bu, bv)


class Operators:
    """All assembled operators for one grid / body / (nu, dt)."""

    def __init__(self, grid, E, nu, dt, pin=0, bn_order=1):
        if bn_order < 1:
            raise ValueError("bn_order must be >= 1")
        self.grid = grid
        self.bn_order = int(bn_order)
        self.nu = float(nu)
        self.dt = float(dt)
        self.E = E.tocsr()
        self.nb = E.shape[0] // 2
        Rd = grid.R_diag()
        Md = grid.M_diag()
        self.Rd = Rd
        self.Md = Md
        self.Mf = Md / Rd                                  # diagonal of M R^{-1}
        self.D = divergence(grid)
        self.G = gradient(grid)
        self.Lhat = laplacian_hat(grid)
        self.L = (sp.diags(Md) @ self.Lhat @ sp.diags(1.0 / Rd)).tocsr()
        self.A = (sp.diags(self.Mf / self.dt) - 0.5 * self.nu * self.L).tocsr()
        self.B1 = self.dt / self.Mf                        # diagonal of B^1 = dt Mf^{-1}
        self.B = bn_matrix(self.B1, self.L, self.nu, self.dt, self.bn_order)
        self.Q = sp.hstack([self.G, self.E.T], format="csr")
        K = (self.Q.T @ self.B @ self.Q).tocsr()
        self.K_unpinned = K
        self.pin = pin
        self.K = pin_matrix(K, pin)
        self.n_q = grid.n_q
        self.n_lambda = grid.n_cell + 2 * self.nb

    def apply_A(self, x):
        return self.A @ x

    def apply_B(self, x):
        return self.B @ x

    def apply_K(self, x):
        return self.K @ x


def bn_matrix(B1, L, nu, dt, order):
    """B^N as a sparse matrix: the first `order` terms of the Neumann series
    dt Mf^{-1} sum_k ((nu dt/2) L Mf^{-1})^k, with B1 the diagonal dt Mf^{-1}.
    Each term is the previous one times (nu dt/2) L Mf^{-1} = (nu/2) L B^1
    from the right, so every term (and the sum) is symmetric when L is."""
    Bd = sp.diags(B1).tocsr()
    term = Bd
    total = Bd
    step = (0.5 * nu * L @ Bd).tocsr()
    for _ in range(order - 1):
        term = (term @ step).tocsr()
        total = (total + term).tocsr()
    total.sort_indices()
    return total


def pin_matrix(K, p):
    """Clear row p and column p of K except the diagonal entry."""
    K = K.tocoo()
    keep = ((K.row != p) & (K.col != p)) | ((K.row == p) & (K.col == p))
    out = sp.csr_matrix((K.data[keep], (K.row[keep], K.col[keep])), shape=K.shape)
    out.eliminate_zeros()
    out.sort_indices()
    return out
