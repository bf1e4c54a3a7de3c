"""The method on a three-dimensional staggered grid (the paper's stated next
step, Sec. 7: a 7-point pressure stencil): the operators of Eqs. 8-11 and
the linear algebra of one time step, Eq. 11 -- the velocity solve, the
modified Poisson solve and the projection -- for given right-hand sides.

Oracle code: test infrastructure only.

The two-dimensional readings carry over axis by axis (x fastest, then y,
then z):
  u_{i,j,k} at (x_i, yc_j, zc_k), i = 1..nx-1   ((nx-1) ny nz values)
  v_{i,j,k} at (xc_i, y_j, zc_k), j = 1..ny-1   (nx (ny-1) nz values)
  w_{i,j,k} at (xc_i, yc_j, z_k), k = 1..nz-1   (nx ny (nz-1) values)
  R = diag(dy_j dz_k | dx_i dz_k | dx_i dy_j)   q = R u, the face fluxes
  M = diag(Dx_i | Dy_j | Dz_k)                  momentum row weights
  Mf = M R^-1, L = M Lhat R^-1, A = Mf/dt - (nu/2) L, B^1 = dt Mf^-1
  D the interior-face divergence, G = -D^T, Q = [G, E^T], K = Q^T B^1 Q
  E = Ehat R^-1, Ehat_{k,f} = (control volume of f) d_h d_h d_h (Eqs. 6-7
  with the product of three one-dimensional deltas); rows 0..nb-1 take u,
  nb..2nb-1 v, 2nb..3nb-1 w; lambda = (phi, f~) with 3 nb forces
  one pressure value pinned: cell (0,0,0), row and column cleared but the
  diagonal.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import delta as delta2
from . import solvers


class Grid3:
    """Metrics of a tensor-product staggered grid in three dimensions."""

    def __init__(self, xf, yf, zf):
        self.f = [np.asarray(a, dtype=np.float64) for a in (xf, yf, zf)]
        self.n = [len(a) - 1 for a in self.f]
        if min(self.n) < 2:
            raise ValueError("need at least 2 cells per direction")
        self.w = [np.diff(a) for a in self.f]                       # cell widths
        if any(np.any(w <= 0) for w in self.w):
            raise ValueError("faces must be strictly increasing")
        self.c = [0.5 * (a[:-1] + a[1:]) for a in self.f]          # cell centres
        self.D = []                                                 # centre-to-centre gaps
        for w in self.w:
            g = np.empty(len(w) + 1)
            g[0] = 0.5 * w[0]
            g[1:-1] = 0.5 * (w[:-1] + w[1:])
            g[-1] = 0.5 * w[-1]
            self.D.append(g)
        nx, ny, nz = self.n
        self.n_comp = [(nx - 1) * ny * nz, nx * (ny - 1) * nz, nx * ny * (nz - 1)]
        self.off = [0, self.n_comp[0], self.n_comp[0] + self.n_comp[1]]
        self.n_q = sum(self.n_comp)
        self.n_cell = nx * ny * nz

    def comp_shape(self, a):
        """(nz, ny, nx) counts of component a's unknowns (x fastest)."""
        s = [self.n[2], self.n[1], self.n[0]]
        s[2 - a] -= 1
        return tuple(s)

    def cidx(self, i, j, k):
        nx, ny, _ = self.n
        return (np.asarray(k) * ny + np.asarray(j)) * nx + np.asarray(i)

    def qidx(self, a, i, j, k):
        """flat index of component a at (i, j, k); the component's own index
        runs 1..n-1, the others 0..n-1."""
        nz, ny, nx = self.comp_shape(a)
        idx = [np.asarray(i), np.asarray(j), np.asarray(k)]
        idx[a] = idx[a] - 1
        return self.off[a] + (idx[2] * ny + idx[1]) * nx + idx[0]

    def _per_face(self, vals_by_axis, a):
        """Tensor product over component a's unknowns of per-axis arrays."""
        vz, vy, vx = vals_by_axis[2], vals_by_axis[1], vals_by_axis[0]
        return (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).ravel()

    def R_diag(self):
        """face areas: dy dz on u, dx dz on v, dx dy on w."""
        one = [np.ones(n) for n in self.n]
        out = []
        for a in range(3):
            axes = []
            for b in range(3):
                if b == a:
                    axes.append(np.ones(self.n[b] - 1))
                else:
                    axes.append(self.w[b])
            out.append(self._per_face(axes, a))
        del one
        return np.concatenate(out)

    def M_diag(self):
        """centre-to-centre gap across the face: Dx on u, Dy on v, Dz on w."""
        out = []
        for a in range(3):
            axes = []
            for b in range(3):
                axes.append(self.D[b][1:-1] if b == a else np.ones(self.n[b]))
            out.append(self._per_face(axes, a))
        return np.concatenate(out)

    def volume_diag(self):
        """control volume of each face unknown: Dx dy dz (u), dx Dy dz (v),
        dx dy Dz (w)."""
        out = []
        for a in range(3):
            axes = []
            for b in range(3):
                axes.append(self.D[b][1:-1] if b == a else self.w[b])
            out.append(self._per_face(axes, a))
        return np.concatenate(out)


def divergence(g):
    """D (n_cell x n_q): the sum over each cell's interior faces of the
    outward flux."""
    nx, ny, nz = g.n
    K, J, I = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    c = g.cidx(I, J, K)
    rows, cols, vals = [], [], []
    for a in range(3):
        idx = [I, J, K]
        # the face on the high side of the cell: index + 1 along a, interior if < n
        hi = [I.copy(), J.copy(), K.copy()]
        hi[a] = idx[a] + 1
        m = hi[a] <= g.n[a] - 1
        rows.append(c[m]); cols.append(g.qidx(a, hi[0][m], hi[1][m], hi[2][m])); vals.append(np.ones(m.sum()))
        m = idx[a] >= 1
        rows.append(c[m]); cols.append(g.qidx(a, I[m], J[m], K[m])); vals.append(-np.ones(m.sum()))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.n_cell, g.n_q))


def _second_difference(centre_gap, left_gap, right_gap):
    n = len(centre_gap)
    lo = 1.0 / (left_gap * centre_gap)
    hi = 1.0 / (right_gap * centre_gap)
    return sp.diags([lo[1:], -(lo + hi), hi[:-1]], [-1, 0, 1], shape=(n, n), format="csr")


def laplacian_hat(g):
    """Lhat on the interior velocity unknowns: per component the sum of the
    three 3-point second differences (7 points), wall neighbours dropped."""
    blocks = []
    for a in range(3):
        ops1 = []
        for b in range(3):
            if b == a:
                # nodes on the face lines 1..n-1, gaps = cell widths
                ops1.append(_second_difference(g.D[b][1:-1], g.w[b][:-1], g.w[b][1:]))
            else:
                # nodes at cell centres, gaps = centre-to-centre distances
                ops1.append(_second_difference(g.w[b], g.D[b][:-1], g.D[b][1:]))
        Ix = sp.identity(ops1[0].shape[0])
        Iy = sp.identity(ops1[1].shape[0])
        Iz = sp.identity(ops1[2].shape[0])
        L = (sp.kron(Iz, sp.kron(Iy, ops1[0])) + sp.kron(Iz, sp.kron(ops1[1], Ix)) +
             sp.kron(ops1[2], sp.kron(Iy, Ix)))
        blocks.append(L)
    return sp.block_diag(blocks, format="csr")


def interpolation_matrix(g, xb, yb, zb):
    """E (3 nb x n_q), flux form, from the product of three deltas (Eq. 6)."""
    xb, yb, zb = (np.asarray(a, dtype=np.float64) for a in (xb, yb, zb))
    nb = len(xb)
    P = [xb, yb, zb]
    rows, cols, vals = [], [], []
    vol = g.volume_diag()
    # positions of each component's unknowns along each axis
    for p in range(nb):
        h = [delta2._local_h(g.f[b], g.w[b], P[b][p], "xyz"[b]) for b in range(3)]
        for a in range(3):
            pos = [g.f[b][1:-1] if b == a else g.c[b] for b in range(3)]
            near = [np.nonzero(np.abs(pos[b] - P[b][p]) < 1.5 * h[b])[0] for b in range(3)]
            for kk in near[2]:
                for jj in near[1]:
                    for ii in near[0]:
                        idx = [ii, jj, kk]
                        full = [idx[b] + 1 if b == a else idx[b] for b in range(3)]
                        f = int(g.qidx(a, full[0], full[1], full[2]))
                        d = 1.0
                        for b in range(3):
                            d *= delta2.delta_h(pos[b][idx[b]] - P[b][p], h[b])
                        rows.append(a * nb + p)
                        cols.append(f)
                        vals.append(vol[f] * d)
    E_hat = sp.csr_matrix((vals, (rows, cols)), shape=(3 * nb, g.n_q))
    return (E_hat @ sp.diags(1.0 / g.R_diag())).tocsr()


def pin_matrix(K, p):
    K = K.tocoo()
    keep = ((K.row != p) & (K.col != p)) | ((K.row == p) & (K.col == p))
    out = sp.csr_matrix((K.data[keep], (K.row[keep], K.col[keep])), shape=K.shape)
    out.eliminate_zeros()
    out.sort_indices()
    return out


class Operators3:
    def __init__(self, g, E, nu, dt, pin=0):
        self.grid = g
        self.nu, self.dt = float(nu), float(dt)
        self.E = E.tocsr()
        self.nb = E.shape[0] // 3
        self.Rd = g.R_diag()
        self.Md = g.M_diag()
        self.Mf = self.Md / self.Rd
        self.D = divergence(g)
        self.G = (-self.D.T).tocsr()
        self.Lhat = laplacian_hat(g)
        self.L = (sp.diags(self.Md) @ self.Lhat @ sp.diags(1.0 / self.Rd)).tocsr()
        self.A = (sp.diags(self.Mf / self.dt) - 0.5 * self.nu * self.L).tocsr()
        self.B1 = self.dt / self.Mf
        self.Q = sp.hstack([self.G, self.E.T], format="csr")
        K = (self.Q.T @ sp.diags(self.B1) @ self.Q).tocsr()
        self.K_unpinned = K
        self.pin = pin
        self.K = pin_matrix(K, pin)
        self.n_q = g.n_q
        self.n_lambda = g.n_cell + 3 * self.nb

    def poisson_rhs(self, qstar, r2):
        """Q^T q* - r2 (Eq. 11b), the pinned entry cleared."""
        rhs = self.Q.T @ qstar - r2
        rhs[self.pin] = 0.0
        return rhs

    def project(self, qstar, lam):
        """q = q* - B^1 Q lambda (Eq. 11c)."""
        return qstar - self.B1 * (self.Q @ lam)


def linear_step(ops, r1, r2, q0, lam0, vel_rtol, poisson_rtol, maxit=20000, hierarchy=None):
    """Eq. 11 for given right-hand sides: A q* = r1 (Jacobi-PCG from q0),
    K lambda = Q^T q* - r2 (AMG-PCG from lam0 with the given hierarchy, else
    Jacobi-PCG), q = q* - B^1 Q lambda.  Returns (q, lambda, q*)."""
    dinv = 1.0 / ops.A.diagonal()
    qs, _, _ = solvers.pcg(lambda x: ops.A @ x, r1, q0, lambda r: dinv * r, vel_rtol, maxit)
    rhs = ops.poisson_rhs(qs, r2)
    if hierarchy is None:
        lam, _, _ = solvers.jacobi_pcg(ops.K, rhs, lam0, poisson_rtol, maxit)
    else:
        lam, _, _ = solvers.amg_pcg(hierarchy, ops.K, rhs, lam0, poisson_rtol, maxit)
    return ops.project(qs, lam), lam, qs
