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
    return sorted(set(re.findall(r"\b(ibpm(?:3d)?_[A-Za-z_0-9]+)\s*\(", text)))


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
    fields = re.findall(r"\b(?:int32_t|double|const double)\s*\*?\s*([a-z_0-9*, \[\]]+);", body)
    flat = []
    for f in fields:
        flat += [x.strip().lstrip("*") for x in f.split(",")]
    names = [re.sub(r"\[\d+\]", "", x) for x in flat]
    assert names == [k for k, _ in ibpm.Params._fields_]
    # the array members keep their lengths
    for x in flat:
        m = re.match(r"([a-z_]+)\[(\d+)\]", x)
        if m:
            ctype = dict(ibpm.Params._fields_)[m.group(1)]
            assert ctype._length_ == int(m.group(2))


def _params(wl, **over):
    return ibpm.make_params(ibpm.params_from_workload(wl, **over))


@pytest.mark.parametrize("over,msg", [
    (dict(bn_order=4), "bn_order must be 1 or 3"),
    (dict(bn_order=2), "bn_order must be 1 or 3"),
    (dict(bn_order=0), "bn_order must be 1 or 3"),
    (dict(bn_order=3, poisson_solver=2), "Jacobi-PCG and AMG-PCG"),
    (dict(bn_order=3, poisson_solver=5), "Jacobi-PCG and AMG-PCG"),
    (dict(poisson_rtol=0.0), "tolerances"),
    (dict(vel_maxit=0), "maxit"),
    (dict(nu=-1.0), "positive"),
    (dict(poisson_solver=7), "solver"),
    (dict(poisson_solver=2, amg_pre=0), "sweep"),
    (dict(poisson_solver=8), "solver"),
    (dict(poisson_solver=4, inner_rtol=1.5), "inner_rtol"),
    (dict(poisson_solver=2, inner_rtol=-1e-3), "inner_rtol"),
    (dict(fuse_transfers=2), "fuse_transfers"),
    (dict(poisson_solver=3, fcg_stall_fall=1.5), "fcg_stall_fall"),
    (dict(poisson_solver=3, fcg_stall_fall=-0.1), "fcg_stall_fall"),
    (dict(bc_kind=(0, 2, 0, 0)), "wall kind"),
    (dict(bc_kind=(1, 0, 0, 0)), "right side only"),
    (dict(bc_kind=(0, 1, 1, 0)), "right side only"),
    (dict(bc_kind=(0, 0, 0, 0), bc_u=(1.0, 0.5, 1.0, 1.0)), "zero net flux"),
    (dict(bc_kind=(0, 1, 0, 0), bc_u=(1.0, 1.0, float("nan"), 1.0)), "finite"),
    (dict(moving_body=2), "moving_body must be 0 or 1"),
    (dict(moving_body=1, bn_order=3), "moving body supports B^1"),
    (dict(moving_body=1, poisson_solver=2), "moving body supports B^1"),
    (dict(moving_body=1, poisson_solver=6), "moving body supports B^1"),
    (dict(moving_body=1, amg_rebuild_every=-1), "amg_rebuild_every"),
    (dict(pin_cell=-1), "pin_cell"),
    (dict(pin_cell=48 * 48), "pin_cell"),
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


def test_paper_re40_grid_supports_are_accepted_on_the_host():
    """Supports that reach the last cell of the uniform patch (the paper's
    Re 40 grid) are accepted; one reaching a stretched cell is not."""
    plan = ibpm.plan_hierarchy(W.cylinder_re40_330())
    assert plan["levels"] >= 2
    wl = W.cylinder_re40_330().replace(xb=np.array([0.515]), yb=np.array([0.0]), ubx=np.zeros(1),
                                       uby=np.zeros(1))
    with pytest.raises(ibpm.IBPMError) as e:
        ibpm.plan_hierarchy(wl)
    assert "uniform" in str(e.value)


def test_null_arguments():
    L = ibpm.load()
    assert L.ibpm_build_operators(None, None, None) == ibpm.IBPM_EINVAL
    assert L.ibpm_last_error(None) == b""
    assert L.ibpm_sizes(None, None, None) == ibpm.IBPM_EINVAL


def test_dirichlet_walls_with_zero_net_flux_are_accepted_on_the_host():
    # all four walls Dirichlet at the freestream: the net flux is zero, so
    # the set-up passes the host checks (the plan call touches no GPU)
    wl = W.cylinder_small(48, 30).replace(poisson_solver=1, bc_kind=(0, 0, 0, 0))
    out = ibpm.plan_hierarchy(wl)
    assert out["levels"] >= 2


@pytest.mark.parametrize("wl", [W.cylinder_small(96, 60).replace(poisson_solver=1),
                                W.cylinder_512()], ids=["96", "512"])
def test_host_hierarchy_matches_the_oracle(wl):
    """The library's host set-up against the oracle's, with no GPU: the same
    level sizes, bit-identical aggregates on the finest level, and the same
    Lanczos spectral-radius estimates (two independent implementations of
    the same steps from the same start vector) to 1e-12."""
    from oracle.problem import Problem
    P = Problem(wl)
    out = ibpm.plan_hierarchy(wl, agg_level=0)
    assert list(out["sizes"]) == P.H.sizes()
    np.testing.assert_array_equal(out["agg"], P.H.levels[0].agg)
    rho_o = np.array([lev.rho for lev in P.H.levels])
    np.testing.assert_allclose(out["rho"], rho_o, rtol=1e-12, atol=0)
    nnz_o = [lev.A.nnz for lev in P.H.levels]
    # the library keeps explicit zeros the oracle's scipy products drop
    assert all(a >= b for a, b in zip(out["nnz"], nnz_o))


def test_pin_cell_moves_the_pinned_row_on_the_host():
    wl = W.cylinder_small(48, 30).replace(poisson_solver=1)
    a = ibpm.plan_hierarchy(wl)
    b = ibpm.plan_hierarchy(wl.replace(pin_cell=47 * 48 + 47))
    assert a["levels"] == b["levels"] and list(a["sizes"])[0] == list(b["sizes"])[0]
    assert a["rho"][0] != b["rho"][0]


@pytest.mark.parametrize("over,msg", [
    (dict(poisson_solver=2), "Jacobi-PCG and AMG-PCG"),
    (dict(vel_rtol=0.0), "tolerances"),
    (dict(nu=-1.0), "positive"),
    (dict(pin_cell=-1), "pin_cell"),
    (dict(amg_pre=0), "sweep"),
])
def test_3d_invalid_parameters_are_rejected_on_the_host(over, msg):
    L = ibpm.load()
    st, keep = ibpm.make_params3(ibpm.params3_from_workload(W.sphere3d(12, radius=0.3), **over))
    h = ctypes.c_void_p()
    rc = L.ibpm3d_build_operators(ctypes.byref(st), None, ctypes.byref(h))
    assert rc == ibpm.IBPM_EINVAL
    assert msg in L.ibpm_last_error(h).decode()
    L.ibpm_destroy(h)


def test_3d_points_outside_the_uniform_cells_are_rejected_on_the_host():
    L = ibpm.load()
    wl = W.sphere3d(12, radius=0.3)
    st, keep = ibpm.make_params3(ibpm.params3_from_workload(wl.replace(zb=wl.zb + 0.9)))
    h = ctypes.c_void_p()
    rc = L.ibpm3d_build_operators(ctypes.byref(st), None, ctypes.byref(h))
    assert rc == ibpm.IBPM_EINVAL
    assert "domain edge" in L.ibpm_last_error(h).decode()
    L.ibpm_destroy(h)


def _defines(prefix):
    text = open(HEADER).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(rf"#define ({prefix}[A-Z_0-9]*)\s+(-?\d+)", text)}


def test_binding_constants_match_the_header():
    """The kernel ids of ibpm_time_kernel / ibpm_iteration_launches, the
    solver ids and the status codes the binding uses are the header's."""
    kern = _defines("IBPM_KERNEL_")
    num = _defines("IBPM_NUM_KERNELS")["IBPM_NUM_KERNELS"]
    assert sorted(kern.values()) == list(range(num))
    assert len(ibpm.KERNELS) == num and sorted(ibpm.KERNELS.values()) == list(range(num))
    for name, k in ibpm.KERNELS.items():
        assert kern["IBPM_KERNEL_" + name.upper()] == k, name
    solvers = _defines("IBPM_SOLVER_")
    for name in ("JACOBI_PCG", "AMG_PCG", "AMG_PCG_MIXED", "AMG_FCG_LEARNED", "AMG_FCG_MIXED_LEARNED",
                 "AMG_PCG_FP32_CYCLE", "AMG_PCG_FP32_CYCLE_GUESS"):
        assert getattr(W, "SOLVER_" + name) == solvers["IBPM_SOLVER_" + name], name
    codes = _defines("IBPM_E")
    codes.update(_defines("IBPM_OK"))
    for name in ("IBPM_OK", "IBPM_EINVAL", "IBPM_ENOMEM", "IBPM_ENOTCONV", "IBPM_EHIP", "IBPM_ENAN"):
        assert getattr(ibpm, name) == codes[name], name
