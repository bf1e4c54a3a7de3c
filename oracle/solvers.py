"""Krylov solvers and the smoothed-aggregation AMG preconditioner (Sec. 3).

Oracle code: test infrastructure only.

Sec. 3 compares CG, diagonally preconditioned CG and CG preconditioned with
smoothed-aggregation algebraic multigrid, and keeps the last.  The paper
names no parameters; the reading used (and matched by the library) is:
  * stop when ||b - K x||_2 <= rtol ||b||_2, measured on the recursively
    updated residual; the true residual is recomputed at exit;
  * strength of connection: j != i with |k_ij| >= max(theta, 1e-12) *
    sqrt(|k_ii k_jj|), theta = 0 by default (the 1e-12 floor only discards
    round-off residue of cancelled entries);
  * aggregation: the three greedy passes of Vanek, Mandel & Brezina in
    natural order -- (1) a node whose strong neighbours are all free roots a
    new aggregate with them, (2) a free node joins the aggregate of its first
    (lowest-index) strong neighbour aggregated in pass 1, (3) a node still
    free roots an aggregate with its free strong neighbours;
  * tentative prolongator T_{i,agg(i)} = 1 (constant near-null space);
  * prolongator P = (I - w D^{-1} K) T with w = 4 / (3 rho), rho an
    estimate of the spectral radius of D^{-1} K: the largest Ritz value of
    LANCZOS_STEPS Lanczos steps on the similar symmetric matrix
    D^{-1/2} K D^{-1/2} (full reorthogonalisation) from a fixed start vector
    (splitmix64 of the unknown index, mapped to [-1/2, 1/2)).  The paper only
    names Cusp's smoothed aggregation, whose Jacobi weights are scaled by
    rho(D^{-1} A); the Gershgorin bound is not used because on the coupled
    system the pressure rows next to force unknowns push it 3-4 times above
    rho, which shrinks every weight by that factor;
  * Galerkin coarse operator P^T K P; coarsen until <= coarse_max unknowns
    or max_levels levels; dense Cholesky on the coarsest level;
  * V-cycle with weighted Jacobi smoothing (weight 4 / (3 rho_level), the
    same estimate),
    `pre` sweeps down and `post` sweeps up, zero initial guess per level.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

STRENGTH_FLOOR = 1e-12
LANCZOS_STEPS = 20


def pcg(apply_A, b, x0, apply_M, rtol, maxit):
    """Preconditioned conjugate gradients.  Returns (x, iterations, true relres)."""
    b = np.asarray(b, dtype=np.float64)
    nb = math.sqrt(float(b @ b))
    if nb == 0.0:
        return np.zeros_like(b), 0, 0.0
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_A(x)
    it = 0
    if math.sqrt(float(r @ r)) > rtol * nb:
        z = apply_M(r)
        p = z.copy()
        rz = float(r @ z)
        while it < maxit:
            it += 1
            Ap = apply_A(p)
            alpha = rz / float(p @ Ap)
            x += alpha * p
            r -= alpha * Ap
            if math.sqrt(float(r @ r)) <= rtol * nb:
                break
            z = apply_M(r)
            rz_new = float(r @ z)
            beta = rz_new / rz
            rz = rz_new
            p = z + beta * p
    rt = b - apply_A(x)
    return x, it, math.sqrt(float(rt @ rt)) / nb


def jacobi_pcg(A, b, x0, rtol, maxit):
    dinv = 1.0 / A.diagonal()
    return pcg(lambda v: A @ v, b, x0, lambda r: dinv * r, rtol, maxit)


# --------------------------------------------------------------------------
# smoothed aggregation
# --------------------------------------------------------------------------

def strength(A, theta):
    """Boolean CSR pattern of strong off-diagonal connections."""
    A = A.tocsr()
    d = A.diagonal()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    vals = A.data
    thr = max(theta, STRENGTH_FLOOR)
    strong = (rows != cols) & (np.abs(vals) >= thr * np.sqrt(np.abs(d[rows] * d[cols])))
    S = sp.csr_matrix((np.ones(strong.sum()), (rows[strong], cols[strong])), shape=A.shape)
    S.sort_indices()
    return S


def aggregate(S):
    """Three-pass greedy aggregation.  Returns (agg array, n_aggregates)."""
    n = S.shape[0]
    ptr, idx = S.indptr, S.indices
    agg = np.full(n, -1, dtype=np.int64)
    nagg = 0
    # pass 1: roots whose whole strong neighbourhood is free
    for i in range(n):
        if agg[i] != -1:
            continue
        nbrs = idx[ptr[i]:ptr[i + 1]]
        if np.all(agg[nbrs] == -1):
            agg[i] = nagg
            agg[nbrs] = nagg
            nagg += 1
    pass1 = agg.copy()
    # pass 2: attach to the first neighbour aggregated in pass 1
    for i in range(n):
        if agg[i] != -1:
            continue
        nbrs = idx[ptr[i]:ptr[i + 1]]
        owners = pass1[nbrs]
        hit = np.nonzero(owners != -1)[0]
        if len(hit):
            agg[i] = owners[hit[0]]
    # pass 3: whatever is left roots aggregates with its free neighbours
    for i in range(n):
        if agg[i] != -1:
            continue
        nbrs = idx[ptr[i]:ptr[i + 1]]
        free = nbrs[agg[nbrs] == -1]
        agg[i] = nagg
        agg[free] = nagg
        nagg += 1
    return agg, nagg


def gershgorin_rho(A):
    """max_i sum_j |a_ij| / |a_ii|, an upper bound of rho(D^{-1} A)."""
    A = A.tocsr()
    rowsum = np.asarray(abs(A).sum(axis=1)).ravel()
    return float(np.max(rowsum / np.abs(A.diagonal())))


def splitmix64_unit(n):
    """Start vector of the Lanczos estimate: entry i is the splitmix64 output
    for the counter i + 1 (Steele, Lea & Flood 2014: add the golden-ratio
    increment, then two xor-shift-multiply rounds and a final xor-shift),
    its top 53 bits scaled to [0, 1), minus 1/2."""
    u64 = np.uint64
    with np.errstate(over="ignore"):
        z = (np.arange(n, dtype=u64) + u64(1)) * u64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> u64(30))) * u64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> u64(27))) * u64(0x94D049BB133111EB)
        z = z ^ (z >> u64(31))
    return (z >> u64(11)).astype(np.float64) / 2.0 ** 53 - 0.5


def lanczos_rho(A, steps=LANCZOS_STEPS):
    """Largest Ritz value of `steps` Lanczos steps on S = D^{-1/2} A D^{-1/2}
    (similar to D^{-1} A, so it has the same eigenvalues), every new vector
    reorthogonalised twice against all earlier ones; the iteration stops
    early when the new vector vanishes (below 1e-12 of |S v|: the Krylov
    space is invariant).  A lower bound of rho(D^{-1} A) that converges to it
    from below."""
    A = A.tocsr()
    n = A.shape[0]
    s = 1.0 / np.sqrt(A.diagonal())
    k = min(steps, n)
    V = np.zeros((k, n))
    alpha = []
    beta = []
    v = splitmix64_unit(n)
    v /= np.linalg.norm(v)
    for j in range(k):
        V[j] = v
        w = s * (A @ (s * v))
        alpha.append(float(v @ w))
        wnorm = float(np.linalg.norm(w))
        for _ in range(2):
            w = w - V[:j + 1].T @ (V[:j + 1] @ w)
        b = float(np.linalg.norm(w))
        if j == k - 1 or b <= 1e-12 * wnorm:
            break
        beta.append(b)
        v = w / b
    T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
    return float(np.linalg.eigvalsh(T)[-1])


class Level:
    def __init__(self, A):
        self.A = A.tocsr()
        self.dinv = 1.0 / self.A.diagonal()
        self.rho = lanczos_rho(self.A)
        self.omega = 4.0 / (3.0 * self.rho)
        self.P = None
        self.agg = None


class SAHierarchy:
    def __init__(self, A, theta=0.0, coarse_max=256, max_levels=12, pre=2, post=2):
        self.pre = pre
        self.post = post
        self.levels = [Level(A)]
        while self.levels[-1].A.shape[0] > coarse_max and len(self.levels) < max_levels:
            lev = self.levels[-1]
            S = strength(lev.A, theta)
            agg, nagg = aggregate(S)
            if nagg >= lev.A.shape[0]:
                break
            n = lev.A.shape[0]
            T = sp.csr_matrix((np.ones(n), (np.arange(n), agg)), shape=(n, nagg))
            w = lev.omega
            P = (T - w * (sp.diags(lev.dinv) @ (lev.A @ T))).tocsr()
            P.sort_indices()
            Ac = (P.T @ lev.A @ P).tocsr()
            Ac.sort_indices()
            lev.P = P
            lev.agg = agg
            self.levels.append(Level(Ac))
        Ac = self.levels[-1].A.toarray()
        self.coarse_chol = sla.cho_factor(Ac, lower=True)

    def refresh(self, A):
        """The hierarchy formed anew for a changed finest operator A (a moving
        body, Sec. 4) with the aggregates and the smoothing weights of this
        set-up kept: each level's P = (I - w D^-1 A) T and Galerkin product
        P^T A P from the new operators, and the coarsest factorisation."""
        self.levels[0].A = A.tocsr()
        for l, lev in enumerate(self.levels):
            lev.dinv = 1.0 / lev.A.diagonal()
            if lev.P is None:
                break
            n = lev.A.shape[0]
            nagg = self.levels[l + 1].A.shape[0]
            T = sp.csr_matrix((np.ones(n), (np.arange(n), lev.agg)), shape=(n, nagg))
            P = (T - lev.omega * (sp.diags(lev.dinv) @ (lev.A @ T))).tocsr()
            P.sort_indices()
            Ac = (P.T @ lev.A @ P).tocsr()
            Ac.sort_indices()
            lev.P = P
            self.levels[l + 1].A = Ac
        Ac = self.levels[-1].A.toarray()
        self.coarse_chol = sla.cho_factor(Ac, lower=True)

    def vcycle(self, b, level=0):
        lev = self.levels[level]
        if level == len(self.levels) - 1:
            return sla.cho_solve(self.coarse_chol, b)
        A, dinv, w = lev.A, lev.dinv, lev.omega
        x = np.zeros_like(b)
        for _ in range(self.pre):
            x = x + w * dinv * (b - A @ x)
        r = b - A @ x
        xc = self.vcycle(lev.P.T @ r, level + 1)
        x = x + lev.P @ xc
        for _ in range(self.post):
            x = x + w * dinv * (b - A @ x)
        return x

    def sizes(self):
        return [lev.A.shape[0] for lev in self.levels]

    def operator_complexity(self):
        return sum(lev.A.nnz for lev in self.levels) / self.levels[0].A.nnz


def amg_pcg(H, A, b, x0, rtol, maxit):
    return pcg(lambda v: A @ v, b, x0, H.vcycle, rtol, maxit)
