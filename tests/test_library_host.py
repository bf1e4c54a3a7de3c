"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid input before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibpm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(ibpm_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_symbols_are_exported():
    L = ibpm.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(ibpm.EXPORTED) == names


def test_param_struct_matches_header_order():
    text = open(HEADER).read()
    body = text[text.index("typedef struct ibpm_params"):text.index("} ibpm_params;")]
    fields = re.findall(r"\b(?:int32_t|double|const double)\s*\*?\s*([a-z_0-9*, ]+);", body)
    flat = []
    for f in fields:
        flat += [x.strip().lstrip("*") for x in f.split(",")]
    assert flat == [k for k, _ in ibpm.Params._fields_]


def _params(wl, **over):
    p = ibpm.params_from_workload(wl, **over)
    st = ibpm.Params()
    keep = []
    for k, _ in ibpm.Params._fields_:
        v = p[k]
        if k in ("xf", "yf", "xb", "yb", "ubx", "uby"):
            a = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
            if a.size == 0:
                a = np.zeros(1)
            keep.append(a)
            setattr(st, k, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        else:
            setattr(st, k, v)
    return st, keep


@pytest.mark.parametrize("over,msg", [
    (dict(bn_order=3), "N = 1"),
    (dict(poisson_rtol=0.0), "tolerances"),
    (dict(vel_maxit=0), "maxit"),
    (dict(nu=-1.0), "positive"),
    (dict(poisson_solver=7), "solver"),
    (dict(poisson_solver=2, amg_pre=0), "sweep"),
    (dict(poisson_solver=6), "solver"),
    (dict(poisson_solver=4, inner_rtol=1.5), "inner_rtol"),
    (dict(poisson_solver=2, inner_rtol=-1e-3), "inner_rtol"),
    (dict(fuse_transfers=2), "fuse_transfers"),
])
def test_invalid_parameters_are_rejected_on_the_host(over, msg):
    L = ibpm.load()
    st, keep = _params(W.cylinder_small(48, 30), **over)
    h = ctypes.c_void_p()
    rc = L.ibpm_build_operators(ctypes.byref(st), None, ctypes.byref(h))
    assert rc == ibpm.IBPM_EINVAL
    assert msg in L.ibpm_last_error(h).decode()
    L.ibpm_destroy(h)


def test_body_on_nonuniform_cells_is_rejected():
    L = ibpm.load()
    wl = W.cylinder_512()
    wl = wl.replace(xb=np.array([0.99]), yb=np.array([0.0]), ubx=np.zeros(1), uby=np.zeros(1))
    st, keep = _params(wl)
    h = ctypes.c_void_p()
    rc = L.ibpm_build_operators(ctypes.byref(st), None, ctypes.byref(h))
    assert rc == ibpm.IBPM_EINVAL
    assert "uniform" in L.ibpm_last_error(h).decode()
    L.ibpm_destroy(h)


def test_null_arguments():
    L = ibpm.load()
    assert L.ibpm_build_operators(None, None, None) == ibpm.IBPM_EINVAL
    assert L.ibpm_last_error(None) == b""
    assert L.ibpm_sizes(None, None, None) == ibpm.IBPM_EINVAL
