"""FP64 reference of the learned preconditioner stage around the network
(an addition to the paper's method; the network itself is in oracle/nn.py).

Oracle code: test infrastructure only.

The stage maps a residual r of the modified Poisson system (Eq. 11b; layout
[pressure cells, x-forces, y-forces]) to a correction e:

  s        = RMS of r over all its entries (1 if r = 0)
  features = 5 images on the cell grid (ny x nx):
             0: pressure residual / s
             1, 2: x- and y-force residuals spread to the cell centres with
                   the delta of Eq. (6), D f / s, where
                   D[c, k] = phi((xc_c - xi_k)/h_x) phi((yc_c - eta_k)/h_y)
                   (h the local cell widths at point k, as for E)
             3, 4: log(dx_i / h_min), log(dy_j / h_min)
  network  = y = N(features) (3 output channels)
  e        = (s / dt) [y_0 on the cells; D^T y_1; D^T y_2]

The 1/dt scaling reflects B^1 = dt M^-1 in K = Q^T B^1 Q, so that
K^-1 r ~ r / dt.

Training loss for a pair (r1, e1) with K e1 = r1 (e1 the error left after
the V-cycle) is the share of the energy-norm error that the correction d
removes when the flexible-CG step scales it optimally:

    loss = -(d . r1)^2 / ((d . K d) (r1 . e1)),   -1 <= loss <= 0

((d . r1)^2 = (d . K e1)^2 <= (d . K d)(e1 . K e1) by Cauchy-Schwarz in the
K inner product, with equality for d parallel to e1).  It weighs the error's
modes by their eigenvalue, so the smooth modes that a local network cannot
represent (and whose amplitude dominates |e1|) do not swamp the ones it can.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import nn
from .delta import _local_h, roma_phi


def cell_delta(grid, xb, yb):
    """D (n_cell x nb, CSR) with the delta weights between cell centres and points."""
    xb = np.asarray(xb, dtype=np.float64)
    yb = np.asarray(yb, dtype=np.float64)
    rows, cols, vals = [], [], []
    for k in range(len(xb)):
        hx = _local_h(grid.xf, grid.dx, xb[k], "x")
        hy = _local_h(grid.yf, grid.dy, yb[k], "y")
        ii = np.nonzero(np.abs(grid.xc - xb[k]) < 1.5 * hx)[0]
        jj = np.nonzero(np.abs(grid.yc - yb[k]) < 1.5 * hy)[0]
        for j in jj:
            for i in ii:
                w = roma_phi((grid.xc[i] - xb[k]) / hx) * roma_phi((grid.yc[j] - yb[k]) / hy)
                rows.append(j * grid.nx + i)
                cols.append(k)
                vals.append(float(w))
    return sp.csr_matrix((vals, (rows, cols)), shape=(grid.nx * grid.ny, len(xb)))


def rms_scale(r):
    r = np.asarray(r, dtype=np.float64)
    s = float(np.sqrt(np.sum(r * r) / r.size)) if r.size else 0.0
    return s if s > 0.0 else 1.0


def features(grid, D, r):
    """(8, ny, nx) input image (channels 5-7 zero) and the scale s."""
    nc, nb = grid.nx * grid.ny, D.shape[1]
    s = rms_scale(r)
    X = np.zeros((8, grid.ny, grid.nx))
    X[0] = (r[:nc] / s).reshape(grid.ny, grid.nx)
    X[1] = (D @ r[nc:nc + nb] / s).reshape(grid.ny, grid.nx)
    X[2] = (D @ r[nc + nb:nc + 2 * nb] / s).reshape(grid.ny, grid.nx)
    hmin = min(grid.dx.min(), grid.dy.min())
    X[3] = np.broadcast_to(np.log(grid.dx / hmin)[None, :], (grid.ny, grid.nx))
    X[4] = np.broadcast_to(np.log(grid.dy / hmin)[:, None], (grid.ny, grid.nx))
    return X, s


def correction(grid, D, y, s, dt):
    """e in lambda layout from the network output y (>= 3 channels)."""
    nc = grid.nx * grid.ny
    yp = y[0].reshape(nc)
    fx = D.T @ y[1].reshape(nc)
    fy = D.T @ y[2].reshape(nc)
    return (s / dt) * np.concatenate([yp, fx, fy])


def energy_loss(d, Kd, r1, e1):
    """-(d.r1)^2 / ((d.Kd)(r1.e1)) and its gradient with respect to d (0 where
    d.Kd <= 0)."""
    a = float(d @ r1)
    b = float(d @ Kd)
    c = float(r1 @ e1)
    if not (b > 0.0) or not (c > 0.0):
        return 0.0, np.zeros_like(d)
    loss = -a * a / (b * c)
    grad = -(2.0 * a / (b * c)) * (r1 - (a / b) * Kd)
    return loss, grad


def correction_adjoint(grid, D, gd, s, dt):
    """Gradient with respect to the network output y of a function of the
    correction e = correction(grid, D, y, s, dt), given its gradient gd."""
    nc, nb = grid.nx * grid.ny, D.shape[1]
    g = np.zeros((3, grid.ny, grid.nx))
    g[0] = (s / dt) * gd[:nc].reshape(grid.ny, grid.nx)
    g[1] = (s / dt) * (D @ gd[nc:nc + nb]).reshape(grid.ny, grid.nx)
    g[2] = (s / dt) * (D @ gd[nc + nb:nc + 2 * nb]).reshape(grid.ny, grid.nx)
    return g


def apply(grid, D, weights, r, dt):
    """e = learned correction of r with the network stored in BF16 (the
    first layer takes the 5 real feature channels)."""
    X, s = features(grid, D, r)
    y = nn.forward_bf16(weights, X[:5])
    return correction(grid, D, y, s, dt)


def sample_loss_grad(grid, D, K, weights, r1, e1, dt):
    """Energy loss of one training pair and the weight gradients (BF16
    storage of weights, activations and back-propagated gradients)."""
    r1 = np.asarray(r1, dtype=np.float64)
    e1 = np.asarray(e1, dtype=np.float64)
    X, s = features(grid, D, r1)
    y, acts = nn.forward_bf16(weights, X[:5], keep=True)
    d = correction(grid, D, y, s, dt)
    loss, gd = energy_loss(d, K @ d, r1, e1)
    dy = np.zeros_like(y)
    dy[:3] = correction_adjoint(grid, D, gd, s, dt)
    return loss, nn.backward_bf16(weights, acts, dy)
