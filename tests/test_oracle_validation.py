"""Validation of the time discretisation against the paper's own numbers,
in the oracle (CPU): the circular Couette flow of Sec. 5.1 (inner cylinder
of radius 0.5 rotated at angular velocity 0.5 inside a fixed one of radius
1, nu = 0.03), whose temporal order of convergence Table 2 (Sec. 5.1) gives
at t = 0.8, 2, 4, 8 for B^1 (0.93-0.99) and for B^3 (2.67-2.85).

The order is log2 of the ratio of the L2 differences between solutions at
time steps dt, dt/2 and dt/2, dt/4 (Sec. 5.1).  The grids are coarser and
the time shorter than the paper's (151^2 to t = 8; here 40^2 and 60^2 to
t = 0.8), so that the oracle finishes in seconds.

With B^1 the first-order splitting error of the projection dominates, and
the impulsive start of the paper gives the paper's order.  With B^3 on this
coarse grid the impulsive start (the body velocity jumps from 0 to its full
value in the first step) brings the order at t = 0.8 down to about 1; with
the rotation brought up smoothly over 0 <= t <= 0.4 (velocity
sin^2(pi t / 0.8) of its full value) the order is about 3.  On the paper's
151^2 grid the impulsive start gives the paper's orders for B^3 too (the GPU
validation tests)."""
import math

import numpy as np
import pytest

from oracle.problem import Problem
from paper_1109_3524_amd import workloads as W


def _run(n, dt, t_end, bn_order, ramp):
    wl = W.couette(n, dt, t_end).replace(bn_order=bn_order, body_ramp=ramp, poisson_maxit=20000)
    P = Problem(wl, vel_rtol=1e-12, poisson_rtol=1e-12)
    st, _ = P.run(wl.nsteps)
    return st.q / P.grid.R_diag()


def _order(n, t_end, bn_order, ramp, dts):
    u = [_run(n, dt, t_end, bn_order, ramp) for dt in dts]
    e1 = np.linalg.norm(u[0] - u[1])
    e2 = np.linalg.norm(u[1] - u[2])
    return math.log2(e1 / e2)


@pytest.mark.timeout(600)
def test_couette_temporal_order_b1_impulsive_start():
    """B^1, impulsive start as in the paper: order 0.97 at t = 0.8 (Table 2
    gives 0.97 at t = 0.8 and 0.93-0.99 overall)."""
    p = _order(40, 0.8, 1, 0.0, (0.02, 0.01, 0.005))
    print(f"B^1 order {p:.3f}")
    assert 0.9 <= p <= 1.05


@pytest.mark.timeout(600)
def test_couette_temporal_order_b3_smooth_start():
    """B^3 with the rotation brought up smoothly: order about 3 (Table 2:
    2.67-2.85 for B^3); with B^1 under the same start the order stays 1,
    so the gain is the B^3 series and not the start."""
    p3 = _order(40, 0.8, 3, 0.4, (0.02, 0.01, 0.005))
    p1 = _order(40, 0.8, 1, 0.4, (0.02, 0.01, 0.005))
    print(f"smooth start: B^3 order {p3:.3f}, B^1 order {p1:.3f}")
    assert 2.6 <= p3 <= 3.2
    assert 0.85 <= p1 <= 1.2


def test_couette_exact_profile():
    """The analytic steady profile of Sec. 5.1: solid-body rotation inside,
    u_theta = Omega r_i at r_i, 0 at r_o, rest outside."""
    ri, ro, om = W.COUETTE_RI, W.COUETTE_RO, W.COUETTE_OMEGA
    for r, ut in ((0.25, om * 0.25), (ri, om * ri), (ro, 0.0), (1.3, 0.0)):
        u, v = W.couette_exact(np.array([0.0]), np.array([r]))
        assert abs(u[0] + ut) < 1e-15 and abs(v[0]) < 1e-15
    r = 0.7
    u, v = W.couette_exact(np.array([r]), np.array([0.0]))
    assert abs(v[0] - om * ri * (ro / r - r / ro) / (ro / ri - ri / ro)) < 1e-15
