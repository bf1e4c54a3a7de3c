"""Synthetic workload generators for the cylinder-flow problems.

This module is the one place both the HIP library and the CPU oracle take
their inputs from.  It holds no arithmetic of the method itself: it only
produces the problem definition (grid face coordinates, Lagrangian point
positions, viscosity, time step, boundary data and solver settings) that
the immersed-boundary projection method then operates on.

The grids follow the recipe of the paper's impulsively started cylinder
runs (Sec. 5.2, Table "gridinfo"): a square domain of side 30 centred on
the body, a uniform patch of width h around the cylinder, and geometric
(exponential) stretching outside it.  The body is a circle of diameter 1
sampled by equally spaced Lagrangian points (Sec. 2, the discussion after
the discrete delta function asks for a spacing close to h).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# Solver selectors shared with the C header (ibpm.h): keep the values equal.
SOLVER_JACOBI_PCG = 0
SOLVER_AMG_PCG = 1
SOLVER_AMG_PCG_MIXED = 2
SOLVER_AMG_FCG_LEARNED = 3
SOLVER_AMG_FCG_MIXED_LEARNED = 4
SOLVER_AMG_PCG_FP32_CYCLE = 5
SOLVER_AMG_PCG_FP32_CYCLE_GUESS = 6

# Wall kinds shared with the C header (ibpm.h), sides ordered left, right,
# bottom, top.
BC_DIRICHLET = 0
BC_CONVECTIVE = 1
PAPER_WALLS = (BC_DIRICHLET, BC_CONVECTIVE, BC_DIRICHLET, BC_DIRICHLET)


def stretch_ratio(n_side: int, h: float, width: float) -> float:
    """Ratio r such that cells h*r, h*r^2, ..., h*r^n_side fill `width`.

    Bisection on the geometric sum; used only to lay out grid faces.
    """
    if n_side <= 0:
        raise ValueError("n_side must be positive")
    if n_side * h >= width:
        raise ValueError("uniform cells already fill the width")
    lo, hi = 1.0, 8.0
    for _ in range(200):
        r = 0.5 * (lo + hi)
        # geometric sum; the log guard avoids overflow of r**n_side for large r
        if n_side * math.log(r) > 700.0:
            s = math.inf
        else:
            s = h * r * (r ** n_side - 1.0) / (r - 1.0)
        if s > width:
            hi = r
        else:
            lo = r
    return 0.5 * (lo + hi)


def uniform_faces(n: int, lo: float, hi: float) -> np.ndarray:
    """n+1 equally spaced face coordinates on [lo, hi]."""
    h = (hi - lo) / n
    k = np.arange(n + 1, dtype=np.float64)
    f = lo + k * h
    f[-1] = hi
    return f


def stretched_faces(n: int, half_domain: float, half_box: float, h: float) -> np.ndarray:
    """Faces of an n-cell line: uniform width h on [-half_box, half_box],
    geometric stretching to +-half_domain outside.  Exactly symmetric
    about 0 (the left half is the mirror image of the right half)."""
    n_uni = int(round(2.0 * half_box / h))
    if (n - n_uni) % 2 != 0 or n_uni % 2 != 0:
        raise ValueError("cell counts must split symmetrically")
    n_side = (n - n_uni) // 2
    r = stretch_ratio(n_side, h, half_domain - half_box)
    half_uni = n_uni // 2
    right = [k * h for k in range(half_uni + 1)]  # 0 .. half_box
    x = right[-1]
    w = h
    for _ in range(n_side):
        w *= r
        x += w
        right.append(x)
    right[-1] = half_domain
    right = np.asarray(right, dtype=np.float64)
    return np.concatenate([-right[:0:-1], right])


def circle_points(n_b: int, cx: float = 0.0, cy: float = 0.0, radius: float = 0.5):
    """n_b equally spaced points on a circle, k = 0 .. n_b-1 counter-clockwise
    from angle 0."""
    th = 2.0 * np.pi * np.arange(n_b, dtype=np.float64) / n_b
    return cx + radius * np.cos(th), cy + radius * np.sin(th)


@dataclasses.dataclass
class Workload:
    """Complete problem definition for one run of the method."""
    name: str
    xf: np.ndarray            # nx+1 x-face coordinates
    yf: np.ndarray            # ny+1 y-face coordinates
    xb: np.ndarray            # n_b Lagrangian x positions
    yb: np.ndarray            # n_b Lagrangian y positions
    ubx: np.ndarray           # n_b prescribed body x-velocity
    uby: np.ndarray           # n_b prescribed body y-velocity
    nu: float                 # kinematic viscosity (U D / Re)
    dt: float                 # time step
    nsteps: int               # steps of the run
    uinf: float = 1.0         # freestream speed
    alpha: float = 0.0        # inflow angle (radians)
    vel_rtol: float = 1e-8    # velocity solve relative residual target
    vel_maxit: int = 2000
    poisson_solver: int = SOLVER_AMG_PCG
    poisson_rtol: float = 1e-8
    poisson_maxit: int = 2000
    amg_theta: float = 0.0    # strength threshold
    amg_pre: int = 2          # pre-smoothing Jacobi sweeps
    amg_post: int = 2         # post-smoothing Jacobi sweeps
    amg_coarse_max: int = 256
    amg_max_levels: int = 12
    pin_cell: int = 0         # pressure cell pinned to 0 (j * nx + i)
    bc_kind: tuple = PAPER_WALLS   # wall kinds, left / right / bottom / top
    bc_u: Optional[tuple] = None   # Dirichlet wall velocities per side;
    bc_v: Optional[tuple] = None   # None: the freestream on every side
    bn_order: int = 1              # N of B^N (the truncated series for A^{-1})
    body_ramp: float = 0.0         # time over which the body velocity rises from rest (sin^2);
                                   # 0: impulsive
    description: str = ""

    def wall_velocities(self):
        """(u, v) per side (left, right, bottom, top): the given Dirichlet
        values, else the freestream (uinf, alpha)."""
        U = self.uinf * math.cos(self.alpha)
        V = self.uinf * math.sin(self.alpha)
        bu = tuple(self.bc_u) if self.bc_u is not None else (U, U, U, U)
        bv = tuple(self.bc_v) if self.bc_v is not None else (V, V, V, V)
        return bu, bv

    @property
    def nx(self) -> int:
        return len(self.xf) - 1

    @property
    def ny(self) -> int:
        return len(self.yf) - 1

    @property
    def nb(self) -> int:
        return len(self.xb)

    @property
    def n_q(self) -> int:
        return (self.nx - 1) * self.ny + self.nx * (self.ny - 1)

    @property
    def n_lambda(self) -> int:
        return self.nx * self.ny + 2 * self.nb

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _body(n_b, cx=0.0, cy=0.0):
    xb, yb = circle_points(n_b, cx, cy)
    return xb, yb, np.zeros(n_b), np.zeros(n_b)


def cylinder_small(n: int = 96, n_b: int = 60, steps: int = 20) -> Workload:
    """2-D flow past a fixed cylinder (D=1), Re=40, uniform n x n grid on
    [-2,2]^2, Jacobi-preconditioned CG for both solves (the small case)."""
    xf = uniform_faces(n, -2.0, 2.0)
    xb, yb, ubx, uby = _body(n_b)
    return Workload(name=f"cylinder_re40_uniform_{n}x{n}", xf=xf, yf=xf.copy(),
                    xb=xb, yb=yb, ubx=ubx, uby=uby, nu=1.0 / 40.0, dt=0.01,
                    nsteps=steps, poisson_solver=SOLVER_JACOBI_PCG,
                    description=f"Re 40 cylinder, uniform {n}^2 on [-2,2]^2, {n_b} points, "
                                "dt 0.01, Jacobi-PCG both solves, rtol 1e-8")


def cylinder_stretched(n: int, h: float, n_b: int, re: float, dt: float, steps: int,
                       cx: float = 0.0, cy: float = 0.0, alpha: float = 0.0,
                       solver: int = SOLVER_AMG_PCG) -> Workload:
    """Cylinder in [-15,15]^2, uniform patch [-1,1]^2 with spacing h, geometric
    stretching outside; n x n cells."""
    xf = stretched_faces(n, 15.0, 1.0, h)
    xb, yb, ubx, uby = _body(n_b, cx, cy)
    return Workload(name=f"cylinder_re{int(re)}_stretched_{n}x{n}", xf=xf, yf=xf.copy(),
                    xb=xb, yb=yb, ubx=ubx, uby=uby, nu=1.0 / re, dt=dt, nsteps=steps,
                    alpha=alpha, poisson_solver=solver,
                    description=f"Re {re:g} cylinder, {n}^2 stretched grid on [-15,15]^2, "
                                f"uniform box [-1,1]^2 h={h}, {n_b} points, dt {dt}")


def cylinder_512(steps: int = 200) -> Workload:
    """The 512^2 Re 40 AMG-PCG workload (262,458 Poisson unknowns)."""
    return cylinder_stretched(512, 0.02, 157, 40.0, 0.005, steps)


def cylinder_1024(steps: int = 500) -> Workload:
    """1024^2 Re 100 workload used for the mixed-precision comparison."""
    return cylinder_stretched(1024, 0.01, 314, 100.0, 0.0025, steps,
                              solver=SOLVER_AMG_PCG_MIXED).replace(poisson_maxit=20000)


def cylinder_2048(steps: int = 2000) -> Workload:
    """2048^2 (4.2M cells) Re 100 workload (the Poisson solve needs a few
    thousand AMG-PCG iterations on this grid)."""
    return cylinder_stretched(2048, 0.005, 628, 100.0, 0.002, steps).replace(poisson_maxit=20000)


def heaving_cylinder(n: int = 512, steps: int = 200) -> Workload:
    """A cylinder in prescribed motion across the stream (a rigid heave, see
    `heave`) on the stretched grids of the fixed-cylinder runs: the 512^2
    (h 0.02, 157 points, dt 0.005), 1024^2 (h 0.01, 314 points, dt 0.0025)
    or 2048^2 (h 0.005, 628 points, dt 0.002) grid at Re 100.  The heave
    keeps the body and its delta supports inside the uniform patch."""
    h, nb, dt = {512: (0.02, 157, 0.005), 1024: (0.01, 314, 0.0025), 2048: (0.005, 628, 0.002)}[n]
    wl = cylinder_stretched(n, h, nb, 100.0, dt, steps).replace(poisson_maxit=20000)
    return wl.replace(name=f"heaving_cylinder_re100_{n}x{n}",
                      description=f"Re 100 cylinder heaving with amplitude {HEAVE_AMPLITUDE} and period "
                                  f"{HEAVE_PERIOD}, {n}^2 stretched grid on [-15,15]^2, h={h}, {nb} points, dt {dt}")


HEAVE_AMPLITUDE = 0.25
HEAVE_PERIOD = 2.0


def heave(wl: Workload, t: float, amplitude: float = HEAVE_AMPLITUDE, period: float = HEAVE_PERIOD):
    """Points and velocities at time t of the workload's body moved as a
    rigid heave y_c(t) = amplitude sin(2 pi t / period): (xb, yb, ubx, uby)."""
    ph = 2.0 * math.pi * t / period
    v = amplitude * (2.0 * math.pi / period) * math.cos(ph)
    return (np.array(wl.xb, dtype=float), np.asarray(wl.yb, dtype=float) + amplitude * math.sin(ph),
            np.zeros(wl.nb), np.full(wl.nb, v))


def cylinder_512_re100(steps: int = 200) -> Workload:
    """512^2 Re 100 grid used for the learned-preconditioner study."""
    return cylinder_stretched(512, 0.02, 157, 100.0, 0.005, steps,
                              solver=SOLVER_AMG_FCG_LEARNED)


COUETTE_RI, COUETTE_RO, COUETTE_OMEGA, COUETTE_NU = 0.5, 1.0, 0.5, 0.03


def couette(n: int, dt: float, t_end: float, solver: int = SOLVER_AMG_PCG) -> Workload:
    """Circular Couette flow (validation of the method): an inner cylinder
    of radius 0.5 impulsively rotated at angular velocity 0.5 inside a fixed
    cylinder of radius 1, both centred at the origin in a fixed square box
    [-1.5,1.5]^2 (side 3: a box of side 1.5 cannot hold the outer cylinder),
    nu = 0.03, fluid at rest at t = 0; uniform n x n grid, points on both
    circles at about the cell width."""
    xf = uniform_faces(n, -1.5, 1.5)
    h = 3.0 / n
    ni = max(8, int(round(2.0 * math.pi * COUETTE_RI / h)))
    no = max(8, int(round(2.0 * math.pi * COUETTE_RO / h)))
    xi, yi = circle_points(ni, radius=COUETTE_RI)
    xo, yo = circle_points(no, radius=COUETTE_RO)
    xb, yb = np.concatenate([xi, xo]), np.concatenate([yi, yo])
    ubx = np.concatenate([-COUETTE_OMEGA * yi, np.zeros(no)])
    uby = np.concatenate([COUETTE_OMEGA * xi, np.zeros(no)])
    steps = int(round(t_end / dt))
    return Workload(name=f"couette_{n}x{n}_dt{dt:g}", xf=xf, yf=xf.copy(), xb=xb, yb=yb,
                    ubx=ubx, uby=uby, nu=COUETTE_NU, dt=dt, nsteps=steps, uinf=0.0,
                    poisson_solver=solver, bc_kind=(BC_DIRICHLET,) * 4,
                    bc_u=(0.0,) * 4, bc_v=(0.0,) * 4,
                    description=f"Couette flow between cylinders r=0.5 (Omega 0.5) and r=1 in "
                                f"[-1.5,1.5]^2, {n}^2 uniform, {ni}+{no} points, nu 0.03, dt {dt:g}, "
                                f"t 0..{t_end:g}")


def couette_exact(x, y):
    """Steady azimuthal velocity of the Couette case as (u, v) at (x, y):
    solid-body rotation inside the inner cylinder, the classical profile
    between the cylinders, rest outside the outer one."""
    r = np.hypot(x, y)
    ri, ro, om = COUETTE_RI, COUETTE_RO, COUETTE_OMEGA
    ut = np.where(r <= ri, om * r,
                  np.where(r <= ro, om * ri * (ro / np.maximum(r, 1e-300) - r / ro) / (ro / ri - ri / ro), 0.0))
    with np.errstate(invalid="ignore", divide="ignore"):
        c = np.where(r > 0, x / np.maximum(r, 1e-300), 0.0)
        s = np.where(r > 0, y / np.maximum(r, 1e-300), 0.0)
    return -ut * s, ut * c


def cylinder_re40_330(steps: int = 10000, dt: float = 0.005) -> Workload:
    """The paper's Re 40 impulsively started cylinder grid (330^2 cells,
    uniform [-0.54,0.54]^2 patch with h = 0.02, geometric stretching to
    [-15,15]^2, about 1.02), 158 points."""
    xf = stretched_faces(330, 15.0, 0.54, 0.02)
    xb, yb, ubx, uby = _body(158)
    return Workload(name="cylinder_re40_stretched_330x330", xf=xf, yf=xf.copy(), xb=xb, yb=yb,
                    ubx=ubx, uby=uby, nu=1.0 / 40.0, dt=dt, nsteps=steps,
                    description="Re 40 cylinder on the paper's 330^2 grid (h 0.02 on [-0.54,0.54]^2, "
                                f"stretched to [-15,15]^2), 158 points, dt {dt:g}")


def harvest_variants(seed: int, count: int = 1) -> List[Dict[str, float]]:
    """Randomised cylinder centres (within +-0.46, keeping the delta support
    inside the uniform patch) and inflow angles (+-10 degrees), seeded."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        cx, cy = rng.uniform(-0.46, 0.46, size=2)
        a = rng.uniform(-10.0, 10.0) * math.pi / 180.0
        out.append({"cx": float(cx), "cy": float(cy), "alpha": float(a)})
    return out


def tiny(nx: int = 12, ny: int = 10, n_b: int = 6, radius: float = 0.25,
         stretched: bool = False, dt: float = 0.01, nu: float = 0.05) -> Workload:
    """Small grids for brute-force dense checks: a body of a few points in
    the middle of a [-1,1]^2 box.  The stretched variant keeps a uniform
    patch [-0.5,0.5]^2 of 8x8 cells (h = 1/8) and stretches the rest out to
    [-1.5,1.5]^2, so nx and ny must be even and at least 10."""
    if stretched:
        xf = stretched_faces(nx, 1.5, 0.5, 0.125)
        yf = stretched_faces(ny, 1.5, 0.5, 0.125)
    else:
        xf, yf = uniform_faces(nx, -1.0, 1.0), uniform_faces(ny, -1.0, 1.0)
    if n_b > 0:
        xb, yb = circle_points(n_b, 0.0, 0.0, radius)
    else:
        xb, yb = np.zeros(0), np.zeros(0)
    return Workload(name=f"tiny_{nx}x{ny}_{n_b}", xf=xf, yf=yf, xb=xb, yb=yb,
                    ubx=np.zeros(n_b), uby=np.zeros(n_b), nu=nu, dt=dt, nsteps=2,
                    poisson_solver=SOLVER_JACOBI_PCG)


def sphere_points(n_b: int, radius: float = 0.5, cx: float = 0.0, cy: float = 0.0, cz: float = 0.0):
    """n_b points spread evenly over a sphere (the golden-angle spiral:
    point k at height 1 - (2k + 1)/n_b, turned by k times the golden
    angle)."""
    k = np.arange(n_b, dtype=np.float64)
    zk = 1.0 - (2.0 * k + 1.0) / n_b
    rk = np.sqrt(np.maximum(0.0, 1.0 - zk * zk))
    th = k * math.pi * (3.0 - math.sqrt(5.0))
    return cx + radius * rk * np.cos(th), cy + radius * rk * np.sin(th), cz + radius * zk


@dataclasses.dataclass
class Workload3:
    """A three-dimensional problem: grid faces, a body's points, and the
    solver settings of one time step's linear algebra (Eq. 11)."""
    name: str
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    xb: np.ndarray
    yb: np.ndarray
    zb: np.ndarray
    nu: float
    dt: float
    vel_rtol: float = 1e-8
    vel_maxit: int = 2000
    poisson_solver: int = SOLVER_AMG_PCG
    poisson_rtol: float = 1e-8
    poisson_maxit: int = 2000
    amg_theta: float = 0.0
    amg_pre: int = 2
    amg_post: int = 2
    amg_coarse_max: int = 256
    amg_max_levels: int = 12
    pin_cell: int = 0
    description: str = ""

    @property
    def nx(self) -> int:
        return len(self.xf) - 1

    @property
    def ny(self) -> int:
        return len(self.yf) - 1

    @property
    def nz(self) -> int:
        return len(self.zf) - 1

    @property
    def nb(self) -> int:
        return len(self.xb)

    @property
    def n_cell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_q(self) -> int:
        nx, ny, nz = self.nx, self.ny, self.nz
        return (nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)

    @property
    def n_lambda(self) -> int:
        return self.n_cell + 3 * self.nb

    def replace(self, **kw) -> "Workload3":
        return dataclasses.replace(self, **kw)


def sphere3d(n: int, n_b: Optional[int] = None, radius: float = 0.5, stretched: bool = False,
             re: float = 100.0, dt: float = 0.01) -> Workload3:
    """A sphere in the box [-1, 1]^3 on an n^3 grid: uniform cells, or (with
    `stretched`) uniform cells of 1/8 on the central n - 2 cells per axis
    and one stretched cell at each end.  n_b points on the sphere (default:
    about one per h^2 of its surface), nu = 2 radius / re."""
    if stretched:
        h = 0.125
        f = stretched_faces(n, 1.0, 0.5 * h * (n - 2), h)
    else:
        f = uniform_faces(n, -1.0, 1.0)
        h = 2.0 / n
    if n_b is None:
        n_b = max(4, int(round(4.0 * math.pi * radius * radius / (h * h))))
    xb, yb, zb = sphere_points(n_b, radius)
    return Workload3(name=f"sphere_re{int(re)}_{'stretched' if stretched else 'uniform'}_{n}^3", xf=f, yf=f.copy(),
                     zf=f.copy(), xb=xb, yb=yb, zb=zb, nu=2.0 * radius / re, dt=dt,
                     description=f"sphere of radius {radius} in [-1,1]^3, {n}^3 cells, {n_b} points, Re {re:g}, "
                                 f"dt {dt}")


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal FP64 vector."""
    return np.random.default_rng(seed).standard_normal(n)


WORKLOADS = {
    "cylinder_small": cylinder_small,
    "cylinder_512": cylinder_512,
    "cylinder_1024": cylinder_1024,
    "cylinder_2048": cylinder_2048,
    "cylinder_512_re100": cylinder_512_re100,
}
