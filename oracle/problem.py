"""Assemble the oracle for one workload and run time steps.

Oracle code: test infrastructure only.
"""
from __future__ import annotations

import math

import numpy as np

from . import delta, flow, operators, solvers
from .grid import Grid

# solver selectors (same numbering as the workload definitions)
JACOBI_PCG = 0
AMG_PCG = 1


class Problem:
    def __init__(self, wl, poisson_solver=None, vel_rtol=None, poisson_rtol=None):
        self.wl = wl
        self.grid = Grid(wl.xf, wl.yf)
        self.E_hat, self.E = delta.interpolation_matrices(self.grid, wl.xb, wl.yb)
        self.ops = operators.Operators(self.grid, self.E, wl.nu, wl.dt, pin=wl.pin_cell,
                                       bn_order=getattr(wl, "bn_order", 1))
        kinds = tuple(wl.bc_kind)
        if any(k not in (flow.BC_DIRICHLET, flow.BC_CONVECTIVE) for k in kinds) or \
                any(k == flow.BC_CONVECTIVE for k in kinds[0:1] + kinds[2:]):
            raise ValueError("wall kinds: Dirichlet anywhere, convective on the right only")
        self.convective = kinds[1] == flow.BC_CONVECTIVE
        self.bc_u, self.bc_v = wl.wall_velocities()
        self.ub = np.concatenate([np.asarray(wl.ubx, float), np.asarray(wl.uby, float)])
        self.solver = wl.poisson_solver if poisson_solver is None else poisson_solver
        self.vel_rtol = wl.vel_rtol if vel_rtol is None else vel_rtol
        self.poisson_rtol = wl.poisson_rtol if poisson_rtol is None else poisson_rtol
        self.H = None
        if self.solver != JACOBI_PCG:
            self.H = solvers.SAHierarchy(self.ops.K, theta=wl.amg_theta,
                                         coarse_max=wl.amg_coarse_max,
                                         max_levels=wl.amg_max_levels,
                                         pre=wl.amg_pre, post=wl.amg_post)

    def move_body(self, xb, yb, ubx, uby, hierarchy="new"):
        """A body in prescribed motion (Sec. 6): the Lagrangian points and
        their velocities at the time the next step advances to.  E and K are
        formed anew for the new positions (the factorised system of Eq. 11 at
        time n+1); the AMG hierarchy is set up anew ("new"), re-formed on the
        aggregates and weights of its first set-up ("refresh"), or re-used
        ("keep", Sec. 4: over several steps) with only its finest level --
        the smoother's operator and diagonal -- following K."""
        wl = self.wl
        self.E_hat, self.E = delta.interpolation_matrices(self.grid, xb, yb)
        self.ops = operators.Operators(self.grid, self.E, wl.nu, wl.dt, pin=wl.pin_cell,
                                       bn_order=getattr(wl, "bn_order", 1))
        self.ub = np.concatenate([np.asarray(ubx, float), np.asarray(uby, float)])
        if hierarchy not in ("new", "refresh", "keep"):
            raise ValueError("hierarchy must be 'new', 'refresh' or 'keep'")
        if self.solver != JACOBI_PCG and hierarchy == "refresh":
            self.H.refresh(self.ops.K)
        elif self.solver != JACOBI_PCG and hierarchy == "keep":
            self.H.levels[0].A = self.ops.K
            self.H.levels[0].dinv = 1.0 / self.ops.K.diagonal()
        elif self.solver != JACOBI_PCG and hierarchy == "new":
            self.H = solvers.SAHierarchy(self.ops.K, theta=wl.amg_theta,
                                         coarse_max=wl.amg_coarse_max,
                                         max_levels=wl.amg_max_levels,
                                         pre=wl.amg_pre, post=wl.amg_post)

    def solve_poisson(self, rhs, x0, rtol=None, maxit=None):
        rtol = self.poisson_rtol if rtol is None else rtol
        maxit = self.wl.poisson_maxit if maxit is None else maxit
        if self.H is None:
            return solvers.jacobi_pcg(self.ops.K, rhs, x0, rtol, maxit)
        return solvers.amg_pcg(self.H, self.ops.K, rhs, x0, rtol, maxit)

    def initial_state(self):
        walls = flow.initial_walls(self.grid, self.wl.bc_kind, self.bc_u, self.bc_v,
                                   self.wl.uinf, self.wl.alpha)
        return flow.initial_state(self.ops, self.wl.uinf, self.wl.alpha, walls)

    def body_velocity(self, step):
        """Prescribed body velocity at the time step `step` advances to: the
        full value, or its sin^2 start-up over the workload's body_ramp."""
        T = getattr(self.wl, "body_ramp", 0.0)
        t = (step + 1) * self.wl.dt
        if T > 0 and t < T:
            return math.sin(0.5 * math.pi * t / T) ** 2 * self.ub
        return self.ub

    def step(self, state):
        return flow.step(self.ops, state, self.body_velocity(state.step), self.wl.uinf, self.wl.alpha,
                         self.vel_rtol, self.wl.vel_maxit, self.solve_poisson,
                         self.convective)

    def run(self, nsteps, state=None, callback=None):
        state = self.initial_state() if state is None else state
        infos = []
        for _ in range(nsteps):
            state, info = self.step(state)
            infos.append(info)
            if callback is not None:
                callback(state, info)
        return state, infos
