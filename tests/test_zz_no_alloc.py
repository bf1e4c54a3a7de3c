"""The allocation-free velocity solve (ibpm_solve_velocity_static) against
the allocating entry point (ibpm_solve_velocity): two calls in a row on one
GPU, the second on a smaller problem, each bit for bit equal to the
allocating solve of the same problem; and the size limit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W

pytestmark = pytest.mark.gpu


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_static_velocity_solve_matches_the_allocating_one():
    # 512^2 (523,264 flux unknowns), then 96^2 (18,240): the array keeps the
    # first call's contents when the second starts
    for wl in (W.cylinder_512(), W.cylinder_small(96, 60)):
        print(f"[static velocity solve] {wl.name} n_q {wl.n_q}", flush=True)
        ctx = ibpm.Context(wl, poisson_solver=0, vel_rtol=1e-12, vel_maxit=5000)
        b = _t(W.random_vector(ctx.n_q, 81))
        x0 = W.random_vector(ctx.n_q, 82)
        q_alloc, q_static = _t(x0), _t(x0)
        s_alloc = ctx.solve_velocity(b, q_alloc)
        s_static = ctx.solve_velocity_static(b, q_static)
        torch.cuda.synchronize()
        print(f"  allocating: {s_alloc['iters']} iters relres {s_alloc['relres']:.3e}; "
              f"static: {s_static['iters']} iters relres {s_static['relres']:.3e}", flush=True)
        assert s_static["status"] == ibpm.IBPM_OK
        assert s_static["iters"] == s_alloc["iters"] and s_static["relres"] == s_alloc["relres"]
        assert torch.equal(q_static, q_alloc)
        # the allocating entry point still works after the static one
        q_again = _t(x0)
        s_again = ctx.solve_velocity(b, q_again)
        assert s_again["iters"] == s_alloc["iters"] and torch.equal(q_again, q_alloc)
        ctx.close()


def test_static_velocity_solve_rejects_grids_beyond_its_array():
    wl = W.cylinder_1024()          # 2,095,104 flux unknowns > 2^20
    ctx = ibpm.Context(wl, poisson_solver=0)
    with pytest.raises(ibpm.IBPMError) as e:
        ctx.solve_velocity_static(ctx.zeros_q(), ctx.zeros_q())
    assert e.value.code == ibpm.IBPM_EINVAL and "exceeds" in str(e.value)
    ctx.close()
