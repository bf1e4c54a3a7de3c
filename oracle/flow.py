"""Boundary values, convection, right-hand sides and one time step of the
immersed-boundary projection method (Sec. 2, Eqs. 3, 8-11; Sec. 5.2 for
the boundary conditions).

Oracle code: test infrastructure only.

One step from (q^n, N(q^{n-1}), lambda^n, walls^n):
  1. walls^{n+1}: Dirichlet walls keep their values (the paper's cylinder
     runs: the freestream on left, bottom, top); a convective outflow
     du/dt + U du/dx = 0 on the right (Sec. 5.2), explicit upwind in time,
     then a uniform shift of the outflow normal velocity so that the net
     flux through the walls is zero (reading: the paper is silent; without
     it the pinned cell would absorb the imbalance).
  2. N(q^n): conservative central differences of div(u u), row-scaled by M.
  3. r1 = (Mf/dt + nu/2 L) q^n + nu/2 (bc_L^n + bc_L^{n+1})
          - 3/2 N(q^n) + 1/2 N(q^{n-1})             (AB2 + Crank-Nicolson)
  4. A q* = r1                                        Eq. (11a)
  5. K lambda = [-D q* + bc2 ; E q* - u_B]           Eq. (11b), r2 = (-bc2, u_B)
  6. q^{n+1} = q* - B^1 Q lambda                      Eq. (11c)
  7. body force F = sum_k f~_k, C_d = 2 F_x, C_l = 2 F_y   (rho = U = D = 1)
Reading for the sign of the force: the matrix form of Eq. (8) puts +E^T f~
on the left of the momentum equation, so the fluid receives -E^T f~ and the
body feels +sum f~.  AB2 start-up: N(q^{-1}) = N(q^0).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import solvers


@dataclasses.dataclass
class Walls:
    """Velocity values on the domain walls.

    uL, uR  (ny)    normal u on the left / right wall at yc_j
    vB, vT  (nx)    normal v on the bottom / top wall at xc_i
    uBt, uTt (nx+1) tangential u on the bottom / top wall at x_i
    vLt, vRt (ny+1) tangential v on the left / right wall at y_j
    """
    uL: np.ndarray
    uR: np.ndarray
    vB: np.ndarray
    vT: np.ndarray
    uBt: np.ndarray
    uTt: np.ndarray
    vLt: np.ndarray
    vRt: np.ndarray

    def copy(self):
        return Walls(*(getattr(self, f.name).copy() for f in dataclasses.fields(self)))


def side_walls(grid, u, v):
    """Walls from one velocity per side, (u, v) each ordered left, right,
    bottom, top: a side's value goes to its normal and tangential entries."""
    nx, ny = grid.nx, grid.ny
    uL, uR, uB, uT = u
    vL, vR, vB, vT = v
    return Walls(uL=np.full(ny, float(uL)), uR=np.full(ny, float(uR)),
                 vB=np.full(nx, float(vB)), vT=np.full(nx, float(vT)),
                 uBt=np.full(nx + 1, float(uB)), uTt=np.full(nx + 1, float(uT)),
                 vLt=np.full(ny + 1, float(vL)), vRt=np.full(ny + 1, float(vR)))


def freestream_walls(grid, uinf, alpha):
    U = uinf * math.cos(alpha)
    V = uinf * math.sin(alpha)
    return side_walls(grid, (U, U, U, U), (V, V, V, V))


BC_DIRICHLET = 0
BC_CONVECTIVE = 1


def initial_walls(grid, kinds, bc_u, bc_v, uinf, alpha):
    """Walls at the start: a Dirichlet side at its (bc_u, bc_v), a convective
    side at the freestream (the initial field, Sec. 5.2)."""
    U = uinf * math.cos(alpha)
    V = uinf * math.sin(alpha)
    u = [U if k == BC_CONVECTIVE else bu for k, bu in zip(kinds, bc_u)]
    v = [V if k == BC_CONVECTIVE else bv for k, bv in zip(kinds, bc_v)]
    return side_walls(grid, u, v)


def velocities(grid, q):
    """u = q^u / dy_j, v = q^v / dx_i as 2-D arrays."""
    qu, qv = grid.split_q(q)
    return qu / grid.dy[:, None], qv / grid.dx[None, :]


def freestream_flux(grid, uinf, alpha):
    U = uinf * math.cos(alpha)
    V = uinf * math.sin(alpha)
    qu = U * np.repeat(grid.dy[:, None], grid.nx - 1, axis=1)
    qv = V * np.repeat(grid.dx[None, :], grid.ny - 1, axis=0)
    return grid.join_q(qu, qv)


def update_walls(grid, walls, q, uinf, alpha, dt, convective=True):
    """walls^n, q^n -> walls^{n+1} (step 1 above).  Without a convective
    (right) wall every wall keeps its value."""
    if not convective:
        return walls.copy()
    u, v = velocities(grid, q)
    Uc = uinf * math.cos(alpha)
    out = walls.copy()
    dxl = grid.dx[-1]
    # normal u on the outflow wall: neighbour u_{nx-1,j} one cell width away
    out.uR = walls.uR - Uc * dt * (walls.uR - u[:, -1]) / dxl
    # tangential v on the outflow wall: neighbour v_{nx-1,j} half a cell away
    out.vRt = walls.vRt.copy()
    out.vRt[1:-1] = walls.vRt[1:-1] - Uc * dt * (walls.vRt[1:-1] - v[:, -1]) / (0.5 * dxl)
    # zero net flux through the walls
    net = (np.sum(out.uR * grid.dy) - np.sum(out.uL * grid.dy)
           + np.sum(out.vT * grid.dx) - np.sum(out.vB * grid.dx))
    out.uR = out.uR - net / np.sum(grid.dy)
    return out


def wall_flux_divergence(grid, walls):
    """Contribution of wall fluxes to the divergence of each cell.

    Full divergence = D q + wall_flux_divergence; bc2 = -wall_flux_divergence
    so that the continuity rows of Eq. (3) read D q = bc2.
    """
    nx, ny = grid.nx, grid.ny
    w = np.zeros((ny, nx))
    w[:, -1] += walls.uR * grid.dy
    w[:, 0] -= walls.uL * grid.dy
    w[-1, :] += walls.vT * grid.dx
    w[0, :] -= walls.vB * grid.dx
    return w.ravel()


def convection(grid, q, walls):
    """N(q): M times central-difference div(u u) on the staggered grid.

    u-momentum at (x_i, yc_j): control volume [xc_{i-1}, xc_i] x [y_j, y_{j+1}]
      M * [ (uc_E^2 - uc_W^2)/Dx_i + ((uv)_N - (uv)_S)/dy_j ]
    v-momentum at (xc_i, y_j): control volume [x_i, x_{i+1}] x [yc_{j-1}, yc_j]
      M * [ ((uv)_E - (uv)_W)/dx_i + (vc_N^2 - vc_S^2)/Dy_j ]
    Cell-centre velocities are means of the two faces; corner velocities
    are distance-weighted linear interpolations across the face line (u in
    y, v in x); corners on a wall take the wall values.  (Reading: the paper
    only says "central differences".)
    """
    nx, ny = grid.nx, grid.ny
    u, v = velocities(grid, q)
    # u including normal wall values: (ny, nx+1), column i <-> x_i
    uf = np.empty((ny, nx + 1))
    uf[:, 0] = walls.uL
    uf[:, -1] = walls.uR
    uf[:, 1:-1] = u
    # v including normal wall values: (ny+1, nx), row j <-> y_j
    vf = np.empty((ny + 1, nx))
    vf[0, :] = walls.vB
    vf[-1, :] = walls.vT
    vf[1:-1, :] = v
    # cell-centre means
    uc = 0.5 * (uf[:, :-1] + uf[:, 1:])          # (ny, nx)
    vc = 0.5 * (vf[:-1, :] + vf[1:, :])          # (ny, nx)
    # corner values at (x_i, y_j), i = 0..nx, j = 0..ny
    ucor = np.zeros((ny + 1, nx + 1))
    vcor = np.zeros((ny + 1, nx + 1))
    ucor[0, :] = walls.uBt
    ucor[-1, :] = walls.uTt
    wlo = (0.5 * grid.dy[1:] / grid.Dy[1:-1])[:, None]   # weight of the row below
    whi = (0.5 * grid.dy[:-1] / grid.Dy[1:-1])[:, None]  # weight of the row above
    ucor[1:-1, :] = wlo * uf[:-1, :] + whi * uf[1:, :]
    vcor[:, 0] = walls.vLt
    vcor[:, -1] = walls.vRt
    wle = (0.5 * grid.dx[1:] / grid.Dx[1:-1])[None, :]   # weight of the column left
    wri = (0.5 * grid.dx[:-1] / grid.Dx[1:-1])[None, :]  # weight of the column right
    vcor[:, 1:-1] = wle * vf[:, :-1] + wri * vf[:, 1:]
    uv = ucor * vcor
    # u-momentum, i = 1..nx-1
    Dx_i = grid.Dx[1:-1][None, :]
    dy_j = grid.dy[:, None]
    Nu = (uc[:, 1:] ** 2 - uc[:, :-1] ** 2) + Dx_i / dy_j * (uv[1:, 1:-1] - uv[:-1, 1:-1])
    # v-momentum, j = 1..ny-1
    Dy_j = grid.Dy[1:-1][:, None]
    dx_i = grid.dx[None, :]
    Nv = Dy_j / dx_i * (uv[1:-1, 1:] - uv[1:-1, :-1]) + (vc[1:, :] ** 2 - vc[:-1, :] ** 2)
    return grid.join_q(Nu, Nv)


def laplacian_full(grid, q, walls):
    """M Lhat u including wall values, by explicit differences (an
    independent evaluation of L q + M bc_L used for the right-hand side)."""
    nx, ny = grid.nx, grid.ny
    u, v = velocities(grid, q)
    dx, dy, Dx, Dy = grid.dx, grid.dy, grid.Dx, grid.Dy
    # u padded: x from wall to wall (nx+1 columns), y with tangential walls (ny+2 rows)
    up = np.empty((ny + 2, nx + 1))
    up[1:-1, 1:-1] = u
    up[1:-1, 0] = walls.uL
    up[1:-1, -1] = walls.uR
    up[0, :] = walls.uBt
    up[-1, :] = walls.uTt
    uc = up[1:-1, 1:-1]
    lap_ux = ((up[1:-1, 2:] - uc) / dx[1:][None, :] - (uc - up[1:-1, :-2]) / dx[:-1][None, :]) / Dx[1:-1][None, :]
    lap_uy = ((up[2:, 1:-1] - uc) / Dy[1:][:, None] - (uc - up[:-2, 1:-1]) / Dy[:-1][:, None]) / dy[:, None]
    Lu = Dx[1:-1][None, :] * (lap_ux + lap_uy)
    vp = np.empty((ny + 1, nx + 2))
    vp[1:-1, 1:-1] = v
    vp[0, 1:-1] = walls.vB
    vp[-1, 1:-1] = walls.vT
    vp[:, 0] = walls.vLt
    vp[:, -1] = walls.vRt
    vc = vp[1:-1, 1:-1]
    lap_vx = ((vp[1:-1, 2:] - vc) / Dx[1:][None, :] - (vc - vp[1:-1, :-2]) / Dx[:-1][None, :]) / dx[None, :]
    lap_vy = ((vp[2:, 1:-1] - vc) / dy[1:][:, None] - (vc - vp[:-2, 1:-1]) / dy[:-1][:, None]) / Dy[1:-1][:, None]
    Lv = Dy[1:-1][:, None] * (lap_vx + lap_vy)
    return grid.join_q(Lu, Lv)


def momentum_rhs(ops, q, conv_now, conv_prev, walls_n, walls_np1):
    """r1 = r^n + bc1 (step 3 above)."""
    from .operators import laplacian_bc
    grid = ops.grid
    nu, dt = ops.nu, ops.dt
    lap_n = laplacian_full(grid, q, walls_n)
    bc_np1 = ops.Md * laplacian_bc(grid, walls_np1)
    return (ops.Mf / dt) * q + 0.5 * nu * (lap_n + bc_np1) - 1.5 * conv_now + 0.5 * conv_prev


def poisson_rhs(ops, qstar, walls_np1, ub):
    """[-D q* + bc2 ; E q* - u_B], pinned entry cleared."""
    grid = ops.grid
    div_full = ops.D @ qstar + wall_flux_divergence(grid, walls_np1)
    rhs = np.concatenate([-div_full, ops.E @ qstar - ub])
    rhs[ops.pin] = 0.0
    return rhs


def project(ops, qstar, lam):
    """q^{n+1} = q* - B^N Q lambda (Eq. 11c), as sparse products."""
    return qstar - ops.apply_B(ops.Q @ lam)


def body_force(ops, lam):
    nc = ops.grid.n_cell
    nb = ops.nb
    return float(np.sum(lam[nc:nc + nb])), float(np.sum(lam[nc + nb:]))


@dataclasses.dataclass
class State:
    q: np.ndarray
    conv_prev: np.ndarray
    lam: np.ndarray
    walls: Walls
    step: int = 0


def initial_state(ops, uinf, alpha, walls=None):
    """Impulsive start: the freestream everywhere, lambda = 0; the walls at
    the freestream unless given."""
    grid = ops.grid
    q = freestream_flux(grid, uinf, alpha)
    if walls is None:
        walls = freestream_walls(grid, uinf, alpha)
    return State(q=q, conv_prev=np.zeros(grid.n_q), lam=np.zeros(ops.n_lambda),
                 walls=walls, step=0)


@dataclasses.dataclass
class StepInfo:
    vel_iters: int
    vel_relres: float
    poisson_iters: int
    poisson_relres: float
    fx: float
    fy: float


def step(ops, state, ub, uinf, alpha, vel_rtol, vel_maxit, poisson_solve, convective=True):
    """Advance one time step.  `poisson_solve(rhs, x0)` -> (x, iters, relres)."""
    grid = ops.grid
    walls_np1 = update_walls(grid, state.walls, state.q, uinf, alpha, ops.dt, convective)
    conv_now = convection(grid, state.q, state.walls)
    conv_prev = conv_now if state.step == 0 else state.conv_prev
    r1 = momentum_rhs(ops, state.q, conv_now, conv_prev, state.walls, walls_np1)
    dinv = 1.0 / ops.A.diagonal()
    qstar, vit, vres = solvers.pcg(ops.apply_A, r1, state.q, lambda r: dinv * r,
                                   vel_rtol, vel_maxit)
    rhs = poisson_rhs(ops, qstar, walls_np1, ub)
    lam, pit, pres = poisson_solve(rhs, state.lam)
    q_new = project(ops, qstar, lam)
    fx, fy = body_force(ops, lam)
    new = State(q=q_new, conv_prev=conv_now, lam=lam, walls=walls_np1, step=state.step + 1)
    return new, StepInfo(vit, vres, pit, pres, fx, fy)
