"""Thin Python binding of the C ABI in include/ibpm.h (ctypes).

Argument marshalling only: every step of the method runs in the HIP kernels
of libibpm.so.  PyTorch provides device memory (float64 CUDA tensors) and
the stream; the library queues all work on the stream that was current
when the context was built.  If the shared library is missing this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibpm.so")

IBPM_OK = 0
IBPM_EINVAL = -1
IBPM_ENOMEM = -2
IBPM_ENOTCONV = -3
IBPM_EHIP = -4
IBPM_ENAN = -5
_CODES = {IBPM_EINVAL: "EINVAL", IBPM_ENOMEM: "ENOMEM", IBPM_ENOTCONV: "ENOTCONV",
          IBPM_EHIP: "EHIP", IBPM_ENAN: "ENAN"}

# every symbol the header declares (checked by the tests)
EXPORTED = (
    "ibpm_build_operators", "ibpm_destroy", "ibpm_last_error", "ibpm_sizes",
    "ibpm_init_state", "ibpm_step", "ibpm_solve_poisson", "ibpm_solve_velocity",
    "ibpm_apply_K", "ibpm_apply_A", "ibpm_stage_walls", "ibpm_stage_rhs1",
    "ibpm_stage_rhs2", "ibpm_stage_project", "ibpm_get_walls", "ibpm_set_walls",
    "ibpm_get_step", "ibpm_set_step", "ibpm_get_forces", "ibpm_hierarchy_info",
    "ibpm_get_aggregates", "ibpm_time_kernel", "ibpm_nn_init", "ibpm_nn_get_weights",
    "ibpm_nn_set_weights", "ibpm_nn_layer", "ibpm_nn_apply", "ibpm_nn_train",
    "ibpm_nn_loss_grad", "ibpm_harvest", "ibpm_plan_hierarchy", "ibpm_iteration_launches",
    "ibpm_nn_adam_step", "ibpm_solve_velocity_static", "ibpm_get_poisson_matrix", "ibpm_bn_info",
    "ibpm_move_body", "ibpm_moving_info", "ibpm3d_build_operators", "ibpm3d_solve_velocity",
    "ibpm3d_apply_A", "ibpm3d_poisson_rhs", "ibpm3d_project", "ibpm3d_linear_step",
)

NN_PARAMS = 39168                     # IBPM_NN_PARAMS
NN_SHAPES = [(32, 5), (32, 32), (32, 32), (32, 32), (32, 32), (3, 32)]   # (out, in) per layer

KERNELS = {"k0_jacobi": 0, "k0_pcg_spmv": 1, "a_pcg_spmv": 2, "k0_residual": 3,
           "restrict0": 4, "prolong0": 5, "pcg_update_k": 6, "coarse_cycle": 7,
           "presmooth0": 8, "stream_copy": 9, "update_presmooth0": 10, "l1_jacobi": 11,
           "copy_level0": 12, "prolong_post0": 13}


class IBPMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("xf", ctypes.POINTER(ctypes.c_double)), ("yf", ctypes.POINTER(ctypes.c_double)),
        ("nb", ctypes.c_int32),
        ("xb", ctypes.POINTER(ctypes.c_double)), ("yb", ctypes.POINTER(ctypes.c_double)),
        ("ubx", ctypes.POINTER(ctypes.c_double)), ("uby", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_double), ("dt", ctypes.c_double),
        ("uinf", ctypes.c_double), ("alpha", ctypes.c_double),
        ("bn_order", ctypes.c_int32),
        ("vel_rtol", ctypes.c_double), ("vel_maxit", ctypes.c_int32),
        ("poisson_solver", ctypes.c_int32), ("poisson_rtol", ctypes.c_double),
        ("poisson_maxit", ctypes.c_int32),
        ("amg_theta", ctypes.c_double), ("amg_pre", ctypes.c_int32), ("amg_post", ctypes.c_int32),
        ("amg_coarse_max", ctypes.c_int32), ("amg_max_levels", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double), ("learned_every", ctypes.c_int32),
        ("fcg_depth", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
        ("fuse_transfers", ctypes.c_int32),
        ("pin_cell", ctypes.c_int32),
        ("bc_kind", ctypes.c_int32 * 4),
        ("bc_u", ctypes.c_double * 4), ("bc_v", ctypes.c_double * 4),
        ("fcg_stall_fall", ctypes.c_double),
        ("body_ramp", ctypes.c_double),
        ("moving_body", ctypes.c_int32),
        ("amg_rebuild_every", ctypes.c_int32),
    ]


class Params3(ctypes.Structure):
    """ibpm3d_params (field order of include/ibpm.h)."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("xf", ctypes.POINTER(ctypes.c_double)), ("yf", ctypes.POINTER(ctypes.c_double)),
        ("zf", ctypes.POINTER(ctypes.c_double)),
        ("nb", ctypes.c_int32),
        ("xb", ctypes.POINTER(ctypes.c_double)), ("yb", ctypes.POINTER(ctypes.c_double)),
        ("zb", ctypes.POINTER(ctypes.c_double)),
        ("nu", ctypes.c_double), ("dt", ctypes.c_double),
        ("vel_rtol", ctypes.c_double), ("vel_maxit", ctypes.c_int32),
        ("poisson_solver", ctypes.c_int32), ("poisson_rtol", ctypes.c_double),
        ("poisson_maxit", ctypes.c_int32),
        ("amg_theta", ctypes.c_double), ("amg_pre", ctypes.c_int32), ("amg_post", ctypes.c_int32),
        ("amg_coarse_max", ctypes.c_int32), ("amg_max_levels", ctypes.c_int32),
        ("pin_cell", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
    ]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres", ctypes.c_double), ("ms", ctypes.c_double),
                ("outer_iters", ctypes.c_int32), ("fallbacks", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("vel_iters", ctypes.c_int32),
                ("poisson_iters", ctypes.c_int32), ("last_vel_iters", ctypes.c_int32),
                ("last_poisson_iters", ctypes.c_int32), ("vel_relres_max", ctypes.c_double),
                ("poisson_relres_max", ctypes.c_double), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("ms", ctypes.c_double),
                ("vel_ms", ctypes.c_double), ("poisson_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Load libibpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1109_3524_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.POINTER(ctypes.c_double)
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "ibpm_build_operators": [ctypes.POINTER(Params), P, ctypes.POINTER(P)],
        "ibpm_destroy": [P],
        "ibpm_sizes": [P, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "ibpm_init_state": [P, P, P, P],
        "ibpm_step": [P, i32, P, P, P, ctypes.POINTER(StepStats)],
        "ibpm_solve_poisson": [P, P, P, ctypes.POINTER(SolveStats)],
        "ibpm_solve_velocity": [P, P, P, ctypes.POINTER(SolveStats)],
        "ibpm_solve_velocity_static": [P, P, P, ctypes.POINTER(SolveStats)],
        "ibpm_apply_K": [P, P, P],
        "ibpm_apply_A": [P, P, P],
        "ibpm_stage_walls": [P, P],
        "ibpm_stage_rhs1": [P, P, P, P, P],
        "ibpm_stage_rhs2": [P, P, P],
        "ibpm_stage_project": [P, P, P, P],
        "ibpm_get_walls": [P, i32, D],
        "ibpm_set_walls": [P, i32, D],
        "ibpm_get_step": [P, ctypes.POINTER(i64)],
        "ibpm_set_step": [P, i64],
        "ibpm_get_forces": [P, D, D],
        "ibpm_hierarchy_info": [P, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "ibpm_get_aggregates": [P, i32, ctypes.POINTER(i32)],
        "ibpm_time_kernel": [P, i32, i32, i64, D, D],
        "ibpm_iteration_launches": [P, i32, ctypes.POINTER(i32)],
        "ibpm_get_poisson_matrix": [P, ctypes.POINTER(i64), P, P, P],
        "ibpm_bn_info": [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                         ctypes.POINTER(i64)],
        "ibpm_move_body": [P, D, D, D, D],
        "ibpm_moving_info": [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)],
        "ibpm3d_build_operators": [ctypes.POINTER(Params3), P, ctypes.POINTER(P)],
        "ibpm3d_solve_velocity": [P, P, P, ctypes.POINTER(SolveStats)],
        "ibpm3d_apply_A": [P, P, P],
        "ibpm3d_poisson_rhs": [P, P, P, P],
        "ibpm3d_project": [P, P, P, P],
        "ibpm3d_linear_step": [P, P, P, P, P, ctypes.POINTER(SolveStats), ctypes.POINTER(SolveStats)],
        "ibpm_nn_init": [P, ctypes.c_uint64],
        "ibpm_nn_get_weights": [P, P, i64],
        "ibpm_nn_set_weights": [P, P, i64],
        "ibpm_nn_layer": [P, i32, i32, P, P, P, P],
        "ibpm_nn_apply": [P, P, P],
        "ibpm_nn_train": [P, P, P, i32, P, i32, i32, ctypes.c_float, D],
        "ibpm_nn_loss_grad": [P, P, P, D, P],
        "ibpm_nn_adam_step": [P, P, ctypes.c_float],
        "ibpm_harvest": [P, P, P, P, i32, P, P, ctypes.POINTER(i32)],
        "ibpm_plan_hierarchy": [ctypes.POINTER(Params), i32, ctypes.POINTER(i32),
                                ctypes.POINTER(i64), ctypes.POINTER(i64), D, i32,
                                ctypes.POINTER(i32), D, ctypes.c_char_p, i32],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.ibpm_last_error.argtypes = [P]
    L.ibpm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params_from_workload(wl: W.Workload, **over) -> dict:
    p = dict(nx=wl.nx, ny=wl.ny, xf=wl.xf, yf=wl.yf, nb=wl.nb, xb=wl.xb, yb=wl.yb,
             ubx=wl.ubx, uby=wl.uby, nu=wl.nu, dt=wl.dt, uinf=wl.uinf, alpha=wl.alpha,
             bn_order=wl.bn_order, vel_rtol=wl.vel_rtol, vel_maxit=wl.vel_maxit,
             poisson_solver=wl.poisson_solver, poisson_rtol=wl.poisson_rtol,
             poisson_maxit=wl.poisson_maxit, amg_theta=wl.amg_theta, amg_pre=wl.amg_pre,
             amg_post=wl.amg_post, amg_coarse_max=wl.amg_coarse_max,
             amg_max_levels=wl.amg_max_levels, inner_rtol=0.0, learned_every=1, fcg_depth=0, use_graphs=1,
             fuse_transfers=1, pin_cell=wl.pin_cell, bc_kind=tuple(wl.bc_kind),
             fcg_stall_fall=0.0, body_ramp=wl.body_ramp, moving_body=0, amg_rebuild_every=0)
    p["bc_u"], p["bc_v"] = wl.wall_velocities()
    p.update(over)
    return p


_ARRAYS = ("xf", "yf", "xb", "yb", "ubx", "uby")


def make_params(p: dict):
    """ibpm_params from a dict of params_from_workload; returns the struct
    and the numpy arrays its pointers refer to (keep them alive)."""
    st = Params()
    keep = {}
    for k, ctype in Params._fields_:
        v = p[k]
        if k in _ARRAYS:
            a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            if a.size == 0:
                a = np.zeros(1)
            keep[k] = a
            setattr(st, k, _dptr(a))
        elif k in ("bc_kind", "bc_u", "bc_v"):
            setattr(st, k, ctype(*v))
        else:
            setattr(st, k, v)
    return st, keep


def plan_hierarchy(wl: W.Workload, agg_level: int = -1, **overrides) -> dict:
    """Host-only set-up of the AMG hierarchy (ibpm_plan_hierarchy): no GPU
    is touched.  Returns sizes, nnz, rho per level, the aggregates of
    `agg_level` (if >= 0) and the host set-up time."""
    L = load()
    st, keep = make_params(params_from_workload(wl, **overrides))
    cap = 32
    nlev = ctypes.c_int32()
    sizes = np.zeros(cap, np.int64)
    nnz = np.zeros(cap, np.int64)
    rho = np.zeros(cap)
    secs = ctypes.c_double()
    err = ctypes.create_string_buffer(512)
    rc = L.ibpm_plan_hierarchy(ctypes.byref(st), cap, ctypes.byref(nlev),
                               sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               nnz.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               _dptr(rho), -1, None, ctypes.byref(secs), err, 512)
    if rc != IBPM_OK:
        raise IBPMError(rc, err.value.decode())
    n = nlev.value
    out = dict(levels=n, sizes=sizes[:n].copy(), nnz=nnz[:n].copy(), rho=rho[:n].copy(),
               seconds=secs.value)
    if agg_level >= 0:
        agg = np.zeros(int(sizes[agg_level]), np.int32)
        rc = L.ibpm_plan_hierarchy(ctypes.byref(st), cap, None, None, None, None, agg_level,
                                   agg.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), None, err, 512)
        if rc != IBPM_OK:
            raise IBPMError(rc, err.value.decode())
        out["agg"] = agg
    return out


class Context:
    """One library context (operators, hierarchy, work memory) on one stream."""

    def __init__(self, wl: W.Workload, **overrides):
        import torch
        self._torch = torch
        L = load()
        p = params_from_workload(wl, **overrides)
        st, self._arrays = make_params(p)
        self.params = p
        self.wl = wl
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = L.ibpm_build_operators(ctypes.byref(st), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h))
        self._h = h
        if rc != IBPM_OK:
            msg = L.ibpm_last_error(h).decode() if h.value else ""
            if h.value:
                L.ibpm_destroy(h)
            self._h = ctypes.c_void_p()
            raise IBPMError(rc, msg)
        nq, nl = ctypes.c_int64(), ctypes.c_int64()
        self._check(L.ibpm_sizes(h, ctypes.byref(nq), ctypes.byref(nl)))
        self.n_q, self.n_lambda = nq.value, nl.value
        self.nx, self.ny, self.nb = wl.nx, wl.ny, wl.nb

    # -- helpers -------------------------------------------------------------
    def _check(self, rc, allow=()):
        if rc != IBPM_OK and rc not in allow:
            raise IBPMError(rc, load().ibpm_last_error(self._h).decode())
        return rc

    def _vec(self, t, n, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be contiguous with {n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def zeros_q(self):
        return self._torch.zeros(self.n_q, dtype=self._torch.float64, device=self.device)

    def zeros_lambda(self):
        return self._torch.zeros(self.n_lambda, dtype=self._torch.float64, device=self.device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ibpm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ---------------------------------------------------------------
    def init_state(self, q=None, conv=None, lam=None):
        q = self.zeros_q() if q is None else q
        conv = self.zeros_q() if conv is None else conv
        lam = self.zeros_lambda() if lam is None else lam
        self._check(load().ibpm_init_state(self._h, self._vec(q, self.n_q, "q"),
                                           self._vec(conv, self.n_q, "conv"),
                                           self._vec(lam, self.n_lambda, "lambda")))
        return q, conv, lam

    def step(self, q, conv, lam, nsteps=1, stats=True, allow_fail=False):
        s = StepStats() if stats else None
        rc = load().ibpm_step(self._h, int(nsteps), self._vec(q, self.n_q, "q"),
                              self._vec(conv, self.n_q, "conv"),
                              self._vec(lam, self.n_lambda, "lambda"),
                              ctypes.byref(s) if s is not None else None)
        self._check(rc, allow=(IBPM_ENOTCONV,) if allow_fail else ())
        return s.as_dict() if s is not None else None

    def solve_poisson(self, rhs, lam, allow_fail=False):
        s = SolveStats()
        rc = load().ibpm_solve_poisson(self._h, self._vec(rhs, self.n_lambda, "rhs"),
                                       self._vec(lam, self.n_lambda, "lambda"), ctypes.byref(s))
        self._check(rc, allow=(IBPM_ENOTCONV, IBPM_ENAN) if allow_fail else ())
        return s.as_dict()

    def solve_velocity(self, rhs, q, allow_fail=False):
        s = SolveStats()
        rc = load().ibpm_solve_velocity(self._h, self._vec(rhs, self.n_q, "rhs"),
                                        self._vec(q, self.n_q, "q"), ctypes.byref(s))
        self._check(rc, allow=(IBPM_ENOTCONV, IBPM_ENAN) if allow_fail else ())
        return s.as_dict()

    def solve_velocity_static(self, rhs, q, allow_fail=False):
        """ibpm_solve_velocity_static: the velocity solve with its work
        memory in the library's static device array (no allocation)."""
        s = SolveStats()
        rc = load().ibpm_solve_velocity_static(self._h, self._vec(rhs, self.n_q, "rhs"),
                                               self._vec(q, self.n_q, "q"), ctypes.byref(s))
        self._check(rc, allow=(IBPM_ENOTCONV, IBPM_ENAN) if allow_fail else ())
        return s.as_dict()

    def apply_K(self, x, y=None):
        y = self.zeros_lambda() if y is None else y
        self._check(load().ibpm_apply_K(self._h, self._vec(x, self.n_lambda, "x"),
                                        self._vec(y, self.n_lambda, "y")))
        return y

    def apply_A(self, x, y=None):
        y = self.zeros_q() if y is None else y
        self._check(load().ibpm_apply_A(self._h, self._vec(x, self.n_q, "x"),
                                        self._vec(y, self.n_q, "y")))
        return y

    def stage_walls(self, q):
        self._check(load().ibpm_stage_walls(self._h, self._vec(q, self.n_q, "q")))

    def stage_rhs1(self, q, conv_prev, r1=None, conv_now=None):
        r1 = self.zeros_q() if r1 is None else r1
        conv_now = self.zeros_q() if conv_now is None else conv_now
        self._check(load().ibpm_stage_rhs1(self._h, self._vec(q, self.n_q, "q"),
                                           self._vec(conv_prev, self.n_q, "conv_prev"),
                                           self._vec(r1, self.n_q, "r1"),
                                           self._vec(conv_now, self.n_q, "conv_now")))
        return r1, conv_now

    def stage_rhs2(self, qstar, rhs=None):
        rhs = self.zeros_lambda() if rhs is None else rhs
        self._check(load().ibpm_stage_rhs2(self._h, self._vec(qstar, self.n_q, "qstar"),
                                           self._vec(rhs, self.n_lambda, "rhs")))
        return rhs

    def stage_project(self, qstar, lam, qout=None):
        qout = self.zeros_q() if qout is None else qout
        self._check(load().ibpm_stage_project(self._h, self._vec(qstar, self.n_q, "qstar"),
                                              self._vec(lam, self.n_lambda, "lambda"),
                                              self._vec(qout, self.n_q, "qout")))
        return qout

    def walls_size(self):
        return 4 * self.nx + 4 * self.ny + 4

    def get_walls(self, which=0):
        out = np.zeros(self.walls_size())
        self._check(load().ibpm_get_walls(self._h, int(which), _dptr(out)))
        return out

    def set_walls(self, which, values):
        a = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
        if a.size != self.walls_size():
            raise ValueError("wrong wall array size")
        self._check(load().ibpm_set_walls(self._h, int(which), _dptr(a)))

    def get_step(self):
        s = ctypes.c_int64()
        self._check(load().ibpm_get_step(self._h, ctypes.byref(s)))
        return s.value

    def set_step(self, step):
        self._check(load().ibpm_set_step(self._h, int(step)))

    def forces(self):
        fx, fy = ctypes.c_double(), ctypes.c_double()
        self._check(load().ibpm_get_forces(self._h, ctypes.byref(fx), ctypes.byref(fy)))
        return fx.value, fy.value

    def hierarchy(self):
        lv = ctypes.c_int32()
        sizes = (ctypes.c_int64 * 64)()
        nnz = (ctypes.c_int64 * 64)()
        self._check(load().ibpm_hierarchy_info(self._h, ctypes.byref(lv), sizes, nnz))
        return [int(sizes[i]) for i in range(lv.value)], [int(nnz[i]) for i in range(lv.value)]

    def time_kernel(self, name, reps=200, min_footprint=0):
        """Mean duration (ms) of one launch of a solver kernel and its
        algorithmic bytes, timed with HIP events on the context's stream;
        min_footprint > 0 rotates the vector operands over copies that span
        at least that many bytes (cold caches)."""
        ms, by = ctypes.c_double(), ctypes.c_double()
        self._check(load().ibpm_time_kernel(self._h, KERNELS[name], int(reps), int(min_footprint),
                                            ctypes.byref(ms), ctypes.byref(by)))
        return ms.value, by.value

    def poisson_matrix(self):
        """The pinned Poisson operator K as the library holds it on the host
        (scipy CSR): for B^N with N > 1 the product formed on the device."""
        import scipy.sparse as sp
        L = load()
        nnz = ctypes.c_int64()
        self._check(L.ibpm_get_poisson_matrix(self._h, ctypes.byref(nnz), None, None, None))
        n = self.n_lambda
        ptr = np.zeros(n + 1, np.int32)
        col = np.zeros(max(nnz.value, 1), np.int32)
        val = np.zeros(max(nnz.value, 1), np.float64)
        self._check(L.ibpm_get_poisson_matrix(self._h, ctypes.byref(nnz), ptr.ctypes.data_as(ctypes.c_void_p),
                                              col.ctypes.data_as(ctypes.c_void_p),
                                              val.ctypes.data_as(ctypes.c_void_p)))
        return sp.csr_matrix((val[:nnz.value], col[:nnz.value], ptr), shape=(n, n))

    def move_body(self, xb, yb, ubx, uby):
        """Move the body's points to (xb, yb) with velocities (ubx, uby) (host
        arrays of nb): E and K are formed anew on the device."""
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (xb, yb, ubx, uby)]
        for a in arrs:
            if a.shape != (self.nb,):
                raise ValueError(f"point arrays must have shape ({self.nb},)")
        self._check(load().ibpm_move_body(self._h, *[_dptr(a) for a in arrs]))

    def moving_info(self):
        """Moves made, hierarchies formed anew, and the cell box E reaches."""
        mv, rf = ctypes.c_int64(), ctypes.c_int64()
        box = (ctypes.c_int32 * 4)()
        self._check(load().ibpm_moving_info(self._h, ctypes.byref(mv), ctypes.byref(rf), box))
        return {"moves": mv.value, "refreshes": rf.value, "box": tuple(int(b) for b in box)}

    def bn_info(self):
        """Stored entries of K and of B^N, and the device memory of the sliced
        triple product (largest slice) against the full intermediate."""
        a, b, c, d = (ctypes.c_int64() for _ in range(4))
        self._check(load().ibpm_bn_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                        ctypes.byref(d)))
        return {"nnz_K": a.value, "nnz_B": b.value, "peak_bytes": c.value, "unsliced_bytes": d.value}

    def iteration_launches(self):
        """Launches per FP64 AMG-PCG iteration of each timeable kernel."""
        cnt = (ctypes.c_int32 * len(KERNELS))()
        self._check(load().ibpm_iteration_launches(self._h, len(KERNELS), cnt))
        return {name: int(cnt[i]) for name, i in KERNELS.items()}

    # -- learned stage ----------------------------------------------------------
    def _f32(self, t, n, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
            raise TypeError(f"{name} must be a float32 CUDA tensor")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be contiguous with {n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def nn_init(self, seed):
        self._check(load().ibpm_nn_init(self._h, ctypes.c_uint64(int(seed))))

    def nn_get_weights(self):
        w = np.zeros(NN_PARAMS, dtype=np.float32)
        self._check(load().ibpm_nn_get_weights(self._h, ctypes.c_void_p(w.ctypes.data), NN_PARAMS))
        return w

    def nn_set_weights(self, w):
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
        if a.size != NN_PARAMS:
            raise ValueError(f"expected {NN_PARAMS} weights")
        self._check(load().ibpm_nn_set_weights(self._h, ctypes.c_void_p(a.ctypes.data), NN_PARAMS))

    def nn_layer(self, layer, mode, x=None, dy=None, mask=None):
        """One network layer on the device (see ibpm_nn_layer); images are
        float32 CUDA tensors of shape (ny, nx, C)."""
        torch = self._torch
        cin = 8 if layer == 0 else 32
        hw = self.nx * self.ny
        xp = self._f32(x, hw * cin, "x") if x is not None else None
        dp = self._f32(dy, hw * 32, "dy") if dy is not None else None
        mp = self._f32(mask, hw * 32, "mask") if mask is not None else None
        if mode == 2:
            co, ci = NN_SHAPES[layer]
            out = torch.zeros(co * ci * 9, dtype=torch.float32, device=self.device)
        else:
            out = torch.zeros(hw * 32, dtype=torch.float32, device=self.device)
        self._check(load().ibpm_nn_layer(self._h, int(layer), int(mode), xp, dp, mp,
                                         ctypes.c_void_p(out.data_ptr())))
        return out

    def nn_apply(self, r, e=None):
        e = self.zeros_lambda() if e is None else e
        self._check(load().ibpm_nn_apply(self._h, self._vec(r, self.n_lambda, "r"),
                                         self._vec(e, self.n_lambda, "e")))
        return e

    def nn_train(self, r1, e1, order, batch, lr):
        """One Adam pass over samples `order` of the (r1, e1) pair set
        (float32 CUDA tensors of shape (nsamples, n_lambda)); returns the mean loss."""
        S = r1.shape[0]
        o = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
        loss = ctypes.c_double()
        self._check(load().ibpm_nn_train(self._h, self._f32(r1, S * self.n_lambda, "r1"),
                                         self._f32(e1, S * self.n_lambda, "e1"), int(S),
                                         ctypes.c_void_p(o.ctypes.data), int(o.size), int(batch),
                                         ctypes.c_float(lr), ctypes.byref(loss)))
        return loss.value

    def nn_adam_step(self, grad, lr):
        """One Adam step on the master weights for a host gradient
        (NN_PARAMS values in the layout of nn_get_weights)."""
        g = np.ascontiguousarray(np.asarray(grad, dtype=np.float32))
        if g.size != NN_PARAMS:
            raise ValueError(f"gradient has {g.size} values, expected {NN_PARAMS}")
        self._check(load().ibpm_nn_adam_step(self._h, g.ctypes.data_as(ctypes.c_void_p), float(lr)))

    def nn_loss_grad(self, r1, e1):
        g = np.zeros(NN_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(load().ibpm_nn_loss_grad(self._h, self._f32(r1, self.n_lambda, "r1"),
                                             self._f32(e1, self.n_lambda, "e1"),
                                             ctypes.byref(loss), ctypes.c_void_p(g.ctypes.data)))
        return loss.value, g

    def harvest(self, rhs, x, xstar, npairs):
        """Training pairs from an AMG-PCG solve started at x (updated in place)."""
        torch = self._torch
        r1 = torch.zeros((npairs, self.n_lambda), dtype=torch.float32, device=self.device)
        e1 = torch.zeros((npairs, self.n_lambda), dtype=torch.float32, device=self.device)
        nout = ctypes.c_int32()
        self._check(load().ibpm_harvest(self._h, self._vec(rhs, self.n_lambda, "rhs"),
                                        self._vec(x, self.n_lambda, "x"),
                                        self._vec(xstar, self.n_lambda, "xstar"), int(npairs),
                                        ctypes.c_void_p(r1.data_ptr()),
                                        ctypes.c_void_p(e1.data_ptr()), ctypes.byref(nout)))
        return r1[:nout.value], e1[:nout.value]

    def aggregates(self, level):
        sizes, _ = self.hierarchy()
        out = np.zeros(sizes[level], dtype=np.int32)
        self._check(load().ibpm_get_aggregates(self._h, int(level),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out


def unpack_walls(w: np.ndarray, nx: int, ny: int) -> dict:
    """Split a packed wall array into its eight parts (layout of ibpm.h)."""
    sizes = [("uL", ny), ("uR", ny), ("vB", nx), ("vT", nx), ("uBt", nx + 1), ("uTt", nx + 1),
             ("vLt", ny + 1), ("vRt", ny + 1)]
    out, o = {}, 0
    for k, n in sizes:
        out[k] = w[o:o + n].copy()
        o += n
    return out


def pack_walls(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[k], dtype=np.float64)
                           for k in ("uL", "uR", "vB", "vT", "uBt", "uTt", "vLt", "vRt")])


def params3_from_workload(wl: W.Workload3, **over) -> dict:
    p = dict(nx=wl.nx, ny=wl.ny, nz=wl.nz, xf=wl.xf, yf=wl.yf, zf=wl.zf, nb=wl.nb, xb=wl.xb, yb=wl.yb,
             zb=wl.zb, nu=wl.nu, dt=wl.dt, vel_rtol=wl.vel_rtol, vel_maxit=wl.vel_maxit,
             poisson_solver=wl.poisson_solver, poisson_rtol=wl.poisson_rtol, poisson_maxit=wl.poisson_maxit,
             amg_theta=wl.amg_theta, amg_pre=wl.amg_pre, amg_post=wl.amg_post, amg_coarse_max=wl.amg_coarse_max,
             amg_max_levels=wl.amg_max_levels, pin_cell=wl.pin_cell, use_graphs=1)
    p.update(over)
    return p


def make_params3(p: dict):
    """ibpm3d_params from a dict of params3_from_workload; returns the struct
    and the numpy arrays its pointers refer to (keep them alive)."""
    st = Params3()
    keep = {}
    for k, _ in Params3._fields_:
        v = p[k]
        if k in ("xf", "yf", "zf", "xb", "yb", "zb"):
            a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            if a.size == 0:
                a = np.zeros(1)
            keep[k] = a
            setattr(st, k, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        else:
            setattr(st, k, v)
    return st, keep


class Context3(Context):
    """A three-dimensional context: the operators of one time step's linear
    algebra (Eq. 11) on the device; the Poisson calls are those of Context."""

    def __init__(self, wl: W.Workload3, **overrides):
        import torch
        self._torch = torch
        L = load()
        p = params3_from_workload(wl, **overrides)
        st, self._arrays = make_params3(p)
        self.params = p
        self.wl = wl
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = L.ibpm3d_build_operators(ctypes.byref(st), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        self._h = h
        if rc != IBPM_OK:
            msg = L.ibpm_last_error(h).decode() if h.value else ""
            if h.value:
                L.ibpm_destroy(h)
            self._h = ctypes.c_void_p()
            raise IBPMError(rc, msg)
        nq, nl = ctypes.c_int64(), ctypes.c_int64()
        self._check(L.ibpm_sizes(h, ctypes.byref(nq), ctypes.byref(nl)))
        self.n_q, self.n_lambda = nq.value, nl.value
        self.nx, self.ny, self.nz, self.nb = wl.nx, wl.ny, wl.nz, wl.nb

    def solve_velocity(self, rhs, q, allow_fail=False):
        s = SolveStats()
        rc = load().ibpm3d_solve_velocity(self._h, self._vec(rhs, self.n_q, "rhs"), self._vec(q, self.n_q, "q"),
                                          ctypes.byref(s))
        self._check(rc, allow=(IBPM_ENOTCONV, IBPM_ENAN) if allow_fail else ())
        return s.as_dict()

    def apply_A(self, x, y=None):
        y = self.zeros_q() if y is None else y
        self._check(load().ibpm3d_apply_A(self._h, self._vec(x, self.n_q, "x"), self._vec(y, self.n_q, "y")))
        return y

    def poisson_rhs(self, qstar, r2, rhs=None):
        rhs = self.zeros_lambda() if rhs is None else rhs
        self._check(load().ibpm3d_poisson_rhs(self._h, self._vec(qstar, self.n_q, "qstar"),
                                              self._vec(r2, self.n_lambda, "r2"),
                                              self._vec(rhs, self.n_lambda, "rhs")))
        return rhs

    def project(self, qstar, lam, qout=None):
        qout = self.zeros_q() if qout is None else qout
        self._check(load().ibpm3d_project(self._h, self._vec(qstar, self.n_q, "qstar"),
                                          self._vec(lam, self.n_lambda, "lambda"),
                                          self._vec(qout, self.n_q, "qout")))
        return qout

    def linear_step(self, r1, r2, q, lam, allow_fail=False):
        sv, sp = SolveStats(), SolveStats()
        rc = load().ibpm3d_linear_step(self._h, self._vec(r1, self.n_q, "r1"), self._vec(r2, self.n_lambda, "r2"),
                                       self._vec(q, self.n_q, "q"), self._vec(lam, self.n_lambda, "lambda"),
                                       ctypes.byref(sv), ctypes.byref(sp))
        self._check(rc, allow=(IBPM_ENOTCONV, IBPM_ENAN) if allow_fail else ())
        return sv.as_dict(), sp.as_dict()
