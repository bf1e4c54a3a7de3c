"""Discrete delta function and the interpolation matrix E (Sec. 2, Eqs. 5-7).

Oracle code: test infrastructure only.

Eq. (6) gives the three-point regularised delta of Roma et al.,
d_h(r) = phi(r/h)/h with
    phi(s) = (5 - 3|s| - sqrt(1 - 3(1-|s|)^2)) / 6   for 0.5 < |s| <= 1.5
    phi(s) = (1 + sqrt(1 - 3 s^2)) / 3               for |s| <= 0.5
    phi(s) = 0                                       otherwise.
Reading: the printed inner interval excludes s = 0, which would make the
kernel vanish at its own centre; it is read as 0 <= |s| <= 0.5 (the two
branches then meet continuously at |s| = 0.5 and phi(0) = 2/3).

Eq. (7): E^_{k,i} = dA_i d_h(x_i - xi_k) d_h(y_i - eta_k), with dA_i the
control area of velocity unknown i.  Reading for the staggered grid: the
control area of u_{i,j} is Dx_i * dy_j and that of v_{i,j} is dx_i * Dy_j
(both equal h^2 on the uniform patch the delta requires).  The matrix that
acts on fluxes is E = E^ R^{-1} (q = R u), so that E q = E^ u is the velocity
interpolated at the Lagrangian points.  Rows 0..nb-1 interpolate u, rows
nb..2nb-1 interpolate v.

The delta needs the grid to be uniform under its support (Sec. 2, text after
Eq. 6); h is the width of the cell holding the point, and every cell within
two cells of it in each direction must have that width (relative 1e-9),
otherwise the point is rejected.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

UNIFORM_RTOL = 1e-9


def roma_phi(s):
    """phi(s) of Eq. (6) for the unit-spaced grid (vectorised)."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    out = np.zeros_like(s)
    inner = s <= 0.5
    outer = (s > 0.5) & (s <= 1.5)
    out[inner] = (1.0 + np.sqrt(1.0 - 3.0 * s[inner] ** 2)) / 3.0
    out[outer] = (5.0 - 3.0 * s[outer] - np.sqrt(1.0 - 3.0 * (1.0 - s[outer]) ** 2)) / 6.0
    return out


def delta_h(r, h):
    """d_h(r) = phi(r/h)/h."""
    return roma_phi(np.asarray(r, dtype=np.float64) / h) / h


def _local_h(faces, widths, x, what):
    """Width h of the cell holding x.  Every cell that meets the open support
    (x - 1.5h, x + 1.5h) must have width h: those are the cells whose widths
    enter the weights (a face inside the support uses the two cells it
    separates, a cell centre inside it its own cell)."""
    i0 = int(np.searchsorted(faces, x, side="right")) - 1
    n = len(widths)
    if i0 < 2 or i0 > n - 3:
        raise ValueError(f"Lagrangian point {what}={x} is too close to the domain edge")
    h = widths[i0]
    first = int(np.searchsorted(faces, x - 1.5 * h, side="right")) - 1
    last = int(np.searchsorted(faces, x + 1.5 * h, side="left")) - 1
    near = widths[first:last + 1]
    if np.any(np.abs(near - h) > UNIFORM_RTOL * h):
        raise ValueError(f"grid is not uniform under the delta support at {what}={x}")
    return h


def interpolation_matrices(grid, xb, yb):
    """Return (E_hat, E) as scipy CSR matrices of shape (2nb, n_q)."""
    xb = np.asarray(xb, dtype=np.float64)
    yb = np.asarray(yb, dtype=np.float64)
    nb = len(xb)
    rows, cols, vals = [], [], []
    # u unknowns: positions x_i (i=1..nx-1), yc_j (j=0..ny-1)
    xu = grid.xf[1:-1]
    yu = grid.yc
    # v unknowns: positions xc_i (i=0..nx-1), y_j (j=1..ny-1)
    xv = grid.xc
    yv = grid.yf[1:-1]
    for k in range(nb):
        hx = _local_h(grid.xf, grid.dx, xb[k], "x")
        hy = _local_h(grid.yf, grid.dy, yb[k], "y")
        # u row k
        iu = np.nonzero(np.abs(xu - xb[k]) < 1.5 * hx)[0]      # offsets into 1..nx-1
        ju = np.nonzero(np.abs(yu - yb[k]) < 1.5 * hy)[0]
        for jj in ju:
            for ii in iu:
                i = ii + 1
                j = jj
                w = grid.Dx[i] * grid.dy[j] * delta_h(xu[ii] - xb[k], hx) * delta_h(yu[jj] - yb[k], hy)
                rows.append(k)
                cols.append(int(grid.uidx(i, j)))
                vals.append(float(w))
        # v row nb+k
        iv = np.nonzero(np.abs(xv - xb[k]) < 1.5 * hx)[0]
        jv = np.nonzero(np.abs(yv - yb[k]) < 1.5 * hy)[0]
        for jj in jv:
            for ii in iv:
                i = ii
                j = jj + 1
                w = grid.dx[i] * grid.Dy[j] * delta_h(xv[ii] - xb[k], hx) * delta_h(yv[jj] - yb[k], hy)
                rows.append(nb + k)
                cols.append(int(grid.vidx(i, j)))
                vals.append(float(w))
    E_hat = sp.csr_matrix((vals, (rows, cols)), shape=(2 * nb, grid.n_q))
    E = (E_hat @ sp.diags(1.0 / grid.R_diag())).tocsr()
    return E_hat, E
