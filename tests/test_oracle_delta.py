"""Pins of the oracle's discrete delta and interpolation matrix against
properties the paper's Eq. (6) and Eq. (7) fix (closed forms, moment
conditions, exactness on uniform and linear fields)."""
import numpy as np
import pytest

from oracle import delta
from oracle.grid import Grid
from paper_1109_3524_amd import workloads as W


def test_delta_closed_form_values():
    phi = delta.roma_phi
    assert phi(0.0) == pytest.approx(2.0 / 3.0, abs=1e-16)
    assert phi(1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert phi(-1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert phi(1.5) == 0.0
    assert phi(2.0) == 0.0
    # both branches give 1/2 at |s| = 0.5 (continuity)
    assert phi(0.5) == pytest.approx(0.5, abs=1e-16)
    assert phi(np.nextafter(0.5, 1.0)) == pytest.approx(0.5, abs=1e-12)
    # d_h scales as 1/h
    assert delta.delta_h(0.0, 0.1) == pytest.approx(20.0 / 3.0)


def test_delta_moment_conditions():
    rng = np.random.default_rng(0)
    s = rng.uniform(0.0, 1.0, size=10000)
    k = np.arange(-3, 4)
    r = s[:, None] - k[None, :]
    w = delta.roma_phi(r)
    np.testing.assert_allclose(w.sum(axis=1), 1.0, atol=2e-15)          # zeroth moment
    np.testing.assert_allclose((r * w).sum(axis=1), 0.0, atol=2e-15)    # first moment
    np.testing.assert_allclose((w * w).sum(axis=1), 0.5, atol=2e-15)    # sum of squares
    # second moment is not constant (quadratics are not interpolated exactly)
    m2 = (r * r * w).sum(axis=1)
    assert m2.max() - m2.min() > 0.05
    assert delta.roma_phi(np.array([0.0]))[0] * 0 + (np.array([-1, 0, 1]) ** 2 * delta.roma_phi(np.array([-1, 0, 1]))).sum() == pytest.approx(1.0 / 3.0)


def _grid_and_E(wl):
    g = Grid(wl.xf, wl.yf)
    Eh, E = delta.interpolation_matrices(g, wl.xb, wl.yb)
    return g, Eh, E


@pytest.mark.parametrize("wl", [W.cylinder_small(48, 30), W.tiny(16, 14, 6, 0.2, stretched=True)])
def test_interpolation_exact_for_uniform_and_linear_fields(wl):
    g, Eh, E = _grid_and_E(wl)
    R = g.R_diag()
    xu, yu = np.meshgrid(g.xf[1:-1], g.yc)
    xv, yv = np.meshgrid(g.xc, g.yf[1:-1])
    nb = wl.nb
    for (a, b, c) in [(1.0, 0.0, 0.0), (0.3, 2.0, -1.5), (-0.7, -0.25, 3.0)]:
        u = a + b * xu + c * yu
        v = 2 * a - c * xv + b * yv
        q = g.join_q(u, v) * R
        interp = E @ q
        np.testing.assert_allclose(interp[:nb], a + b * wl.xb + c * wl.yb, atol=1e-13)
        np.testing.assert_allclose(interp[nb:], 2 * a - c * wl.xb + b * wl.yb, atol=1e-13)
        np.testing.assert_allclose(Eh @ g.join_q(u, v), interp, atol=1e-13)
    # a quadratic is not reproduced exactly (negative check)
    u = xu ** 2
    q = g.join_q(u, 0 * xv) * R
    assert np.max(np.abs((E @ q)[:nb] - wl.xb ** 2)) > 1e-6


def test_spreading_conserves_total_force():
    wl = W.cylinder_small(48, 30)
    g, Eh, E = _grid_and_E(wl)
    f = np.random.default_rng(3).standard_normal(2 * wl.nb)
    spread = E.T @ f
    R = g.R_diag()
    su = np.sum((R * spread)[:g.n_u])
    sv = np.sum((R * spread)[g.n_u:])
    assert su == pytest.approx(f[:wl.nb].sum(), abs=1e-12)
    assert sv == pytest.approx(f[wl.nb:].sum(), abs=1e-12)


def test_support_is_three_by_three():
    wl = W.cylinder_small(96, 60)
    g, Eh, E = _grid_and_E(wl)
    counts = np.diff(E.indptr)
    # Generically 3 nodes per direction lie in |r| < 1.5h.  A point exactly
    # half-way between two nodes has 2, plus up to two nodes at
    # |r| = 1.5h (1 - eps) after rounding, whose weights are O(eps^2).
    assert counts.max() <= 12
    assert counts.min() >= 6
    big = E.data[np.abs(E.data) > 1e-12 * np.abs(E.data).max()]
    assert len(big) <= 9 * 2 * wl.nb


def test_nonuniform_support_rejected():
    wl = W.cylinder_512()
    g = Grid(wl.xf, wl.yf)
    with pytest.raises(ValueError):
        delta.interpolation_matrices(g, np.array([0.99]), np.array([0.0]))
    with pytest.raises(ValueError):
        delta.interpolation_matrices(g, np.array([0.0]), np.array([3.0]))


def test_support_up_to_the_edge_of_the_uniform_patch_is_accepted():
    """The paper's Re 40 grid (Table 3) keeps a uniform patch [-0.54,0.54]
    with h = 0.02 around a cylinder of radius 0.5: the supports reach 0.53,
    inside the patch, and are accepted; a point 0.015 further out has a
    support reaching a stretched cell and is rejected."""
    wl = W.cylinder_re40_330()
    g = Grid(wl.xf, wl.yf)
    _, E = delta.interpolation_matrices(g, wl.xb, wl.yb)
    assert E.shape[0] == 2 * wl.nb
    delta.interpolation_matrices(g, np.array([0.51]), np.array([0.0]))
    with pytest.raises(ValueError):
        delta.interpolation_matrices(g, np.array([0.515]), np.array([0.0]))
