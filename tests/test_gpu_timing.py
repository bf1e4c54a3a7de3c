"""The kernel timer of the library (ibpm_time_kernel) on the 512^2 grid:
every timeable kernel runs on cold operand sets and reports a positive
mean duration and its algorithmic bytes; the level-0 copy moves exactly
two level-0 vectors per launch.  The one-pass prolongation and post-smoothing
is switched on for this grid (it is on by default from 2^22 cells), so the
launch plan names it in place of the separate passes."""
import pytest

torch = pytest.importorskip("torch")

from paper_1109_3524_amd import ibpm
from paper_1109_3524_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_every_timeable_kernel_times_on_cold_operands(monkeypatch):
    monkeypatch.setenv("IBPM_POST_FUSE", "1")
    wl = W.cylinder_512()
    ctx = ibpm.Context(wl, poisson_solver=1)
    plan = ctx.iteration_launches()
    for name in ibpm.KERNELS:
        ms, by = ctx.time_kernel(name, 4, 1 << 28)
        print(f"  {name:18s} {1e3 * ms:8.2f} us {by / 1e6:9.2f} MB launches/iter {plan[name]}", flush=True)
        assert ms > 0 and by > 0
    _, by = ctx.time_kernel("copy_level0", 2)
    assert by == 16.0 * (ctx.n_lambda - ctx.n_lambda % 2)
    assert plan["copy_level0"] == 0 and plan["stream_copy"] == 0
    assert plan["prolong_post0"] == 1 and plan["prolong0"] == 0 and plan["k0_jacobi"] == 0
    ctx.close()
