"""Staggered Cartesian grid metrics (Sec. 2: the equations are discretised
on a staggered, possibly non-uniform Cartesian grid).

Oracle code: test infrastructure only.

Layout of the unknowns (x index fastest everywhere):
  u_{i,j}  at (x_i,  yc_j), i = 1..nx-1, j = 0..ny-1   -> (nx-1)*ny values
  v_{i,j}  at (xc_i, y_j),  i = 0..nx-1, j = 1..ny-1   -> nx*(ny-1) values
  phi_{i,j} at cell centres (xc_i, yc_j)               -> nx*ny values
The flux vector is q = [q^u; q^v] with q^u = u * dy_j and q^v = v * dx_i.
"""
from __future__ import annotations

import numpy as np


class Grid:
    """Metrics of a tensor-product staggered grid given its face lines."""

    def __init__(self, xf, yf):
        self.xf = np.asarray(xf, dtype=np.float64)
        self.yf = np.asarray(yf, dtype=np.float64)
        if self.xf.ndim != 1 or self.yf.ndim != 1:
            raise ValueError("face arrays must be 1-D")
        self.nx = len(self.xf) - 1
        self.ny = len(self.yf) - 1
        if self.nx < 2 or self.ny < 2:
            raise ValueError("need at least 2 cells per direction")
        self.dx = np.diff(self.xf)
        self.dy = np.diff(self.yf)
        if np.any(self.dx <= 0) or np.any(self.dy <= 0):
            raise ValueError("faces must be strictly increasing")
        self.xc = 0.5 * (self.xf[:-1] + self.xf[1:])
        self.yc = 0.5 * (self.yf[:-1] + self.yf[1:])
        # Distance between the two unknowns on either side of face line i
        # (centre-to-centre); at the domain edges it is the half cell from
        # the edge centre to the wall, where tangential wall values sit.
        self.Dx = np.empty(self.nx + 1)
        self.Dx[0] = 0.5 * self.dx[0]
        self.Dx[1:-1] = 0.5 * (self.dx[:-1] + self.dx[1:])
        self.Dx[-1] = 0.5 * self.dx[-1]
        self.Dy = np.empty(self.ny + 1)
        self.Dy[0] = 0.5 * self.dy[0]
        self.Dy[1:-1] = 0.5 * (self.dy[:-1] + self.dy[1:])
        self.Dy[-1] = 0.5 * self.dy[-1]
        self.n_u = (self.nx - 1) * self.ny
        self.n_v = self.nx * (self.ny - 1)
        self.n_q = self.n_u + self.n_v
        self.n_cell = self.nx * self.ny

    # index maps into the flat vectors -------------------------------------
    def uidx(self, i, j):
        """flat index of u_{i,j}, i = 1..nx-1."""
        return np.asarray(j) * (self.nx - 1) + (np.asarray(i) - 1)

    def vidx(self, i, j):
        """flat index of v_{i,j} in q, j = 1..ny-1."""
        return self.n_u + (np.asarray(j) - 1) * self.nx + np.asarray(i)

    def cidx(self, i, j):
        """flat index of cell (i,j)."""
        return np.asarray(j) * self.nx + np.asarray(i)

    # split / join helpers ---------------------------------------------------
    def split_q(self, q):
        """q -> (qu as (ny, nx-1), qv as (ny-1, nx))."""
        q = np.asarray(q)
        return (q[:self.n_u].reshape(self.ny, self.nx - 1),
                q[self.n_u:].reshape(self.ny - 1, self.nx))

    def join_q(self, qu, qv):
        return np.concatenate([np.ravel(qu), np.ravel(qv)])

    def R_diag(self):
        """diagonal of R (q = R u): dy_j on u unknowns, dx_i on v unknowns."""
        ru = np.repeat(self.dy, self.nx - 1)
        rv = np.tile(self.dx, self.ny - 1)
        return np.concatenate([ru, rv])

    def M_diag(self):
        """momentum row scaling M: Dx_i on u rows, Dy_j on v rows."""
        mu = np.tile(self.Dx[1:-1], self.ny)
        mv = np.repeat(self.Dy[1:-1], self.nx)
        return np.concatenate([mu, mv])

    def cell_of(self, faces, x):
        """index i of the cell [faces[i], faces[i+1]) that contains x."""
        i = int(np.searchsorted(faces, x, side="right")) - 1
        return min(max(i, 0), len(faces) - 2)
