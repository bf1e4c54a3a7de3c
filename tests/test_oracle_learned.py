"""Pins of the learned-stage oracle: the cell-centre delta weights against
the moment conditions of the delta of Eq. (6), the feature and output maps
against closed forms, the energy loss against its bounds, optimum and
finite differences, and the BF16-storage network against the FP64 one on
exactly representable values."""
import numpy as np

from oracle import learned, nn
from oracle.grid import Grid
from paper_1109_3524_amd import workloads as W


def _grid(wl):
    return Grid(wl.xf, wl.yf)


def test_cell_delta_partition_of_unity_and_first_moment():
    # on a uniform patch the Roma delta reproduces constants and linear
    # functions exactly: sum_c D[c,k] = 1, sum_c (xc - xi_k) D[c,k] = 0
    wl = W.tiny(40, 36, 9, radius=0.3)
    g = _grid(wl)
    D = learned.cell_delta(g, wl.xb, wl.yb).toarray()
    X, Y = np.meshgrid(g.xc, g.yc)
    X, Y = X.reshape(-1), Y.reshape(-1)
    np.testing.assert_allclose(D.sum(axis=0), 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(((X[:, None] - wl.xb[None, :]) * D).sum(axis=0), 0.0, atol=1e-14)
    np.testing.assert_allclose(((Y[:, None] - wl.yb[None, :]) * D).sum(axis=0), 0.0, atol=1e-14)
    # a point on a cell centre gets the weight phi(0)^2 = 4/9 there
    g2 = Grid(W.uniform_faces(10, 0.0, 1.0), W.uniform_faces(10, 0.0, 1.0))
    D2 = learned.cell_delta(g2, [0.45], [0.55]).toarray()
    assert abs(D2[5 * 10 + 4, 0] - 4.0 / 9.0) < 1e-15
    assert np.count_nonzero(D2) == 9


def test_features_scale_and_geometry_channels():
    wl = W.tiny(20, 18, 6, radius=0.12, stretched=True)
    g = _grid(wl)
    D = learned.cell_delta(g, wl.xb, wl.yb)
    n = g.nx * g.ny + 2 * wl.nb
    r = W.random_vector(n, 3) * 7.5
    X, s = learned.features(g, D, r)
    assert abs(s - np.sqrt(np.mean(r * r))) < 1e-12 * s
    np.testing.assert_allclose(X[0].reshape(-1), r[:g.nx * g.ny] / s, rtol=1e-15)
    # channel 3 depends on the column only and is 0 on the finest cells
    assert np.all(X[3] == X[3][0:1, :])
    assert np.min(np.abs(X[3])) == 0.0 and np.min(X[3]) >= 0.0
    assert np.all(X[4] == X[4][:, 0:1])
    assert np.all(X[5:] == 0.0)
    # scaling r leaves the features unchanged (the scale absorbs it)
    X2, s2 = learned.features(g, D, 1e-6 * r)
    np.testing.assert_allclose(X2, X, rtol=1e-12, atol=1e-15)
    assert learned.rms_scale(np.zeros(5)) == 1.0


def test_correction_reproduces_constant_force_field():
    wl = W.tiny(30, 30, 8, radius=0.35)
    g = _grid(wl)
    D = learned.cell_delta(g, wl.xb, wl.yb)
    y = np.zeros((3, g.ny, g.nx))
    y[0] = np.arange(g.nx * g.ny).reshape(g.ny, g.nx)
    y[1] = 2.0
    y[2] = -3.0
    e = learned.correction(g, D, y, 4.0, 0.5)
    nc = g.nx * g.ny
    np.testing.assert_allclose(e[:nc], 8.0 * np.arange(nc))
    np.testing.assert_allclose(e[nc:nc + 8], 16.0, rtol=1e-14)
    np.testing.assert_allclose(e[nc + 8:], -24.0, rtol=1e-14)


def test_bf16_network_equals_fp64_network_on_representable_values():
    # weights in {-1, 0, 1} and small integer inputs keep every activation an
    # integer below 256, which BF16 holds exactly
    rng = np.random.default_rng(7)
    ws = [rng.integers(-1, 2, size=(4, 2, 3, 3)).astype(float) * (rng.random((4, 2, 3, 3)) < 0.3),
          rng.integers(-1, 2, size=(3, 4, 3, 3)).astype(float) * (rng.random((3, 4, 3, 3)) < 0.3)]
    x = rng.integers(-2, 3, size=(2, 6, 7)).astype(float)
    y, acts = nn.forward_bf16(ws, x, keep=True)
    assert np.max(np.abs(acts[1])) < 256
    np.testing.assert_array_equal(y, nn.forward(ws, x))
    dout = rng.integers(-2, 3, size=y.shape).astype(float)
    for a, b in zip(nn.backward_bf16(ws, acts, dout), nn.backward(ws, nn.forward(ws, x, keep=True)[1], dout)):
        np.testing.assert_array_equal(a, b)
    # general values: agreement to BF16 precision
    ws = nn.init_weights([2, 4, 3], seed=1)
    x = rng.standard_normal((2, 6, 7))
    assert np.linalg.norm(nn.forward_bf16(ws, x) - nn.forward(ws, x)) < 2e-2 * np.linalg.norm(nn.forward(ws, x))


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0])
    out = nn.bf16_round(vals)
    np.testing.assert_array_equal(out, [1.0, 1.0, 1.0 + 2 ** -6 * 1.0, 1.0, -2.5, 0.0])


def test_correction_is_positively_homogeneous_in_the_residual():
    # the features see r / rms(r) and the output is scaled back by rms(r), so
    # doubling r doubles the correction exactly (powers of two are exact)
    wl = W.tiny(14, 12, 6, radius=0.3)
    g = _grid(wl)
    D = learned.cell_delta(g, wl.xb, wl.yb)
    ws = nn.init_weights([5, 8, 8, 3], seed=4)
    r = W.random_vector(g.nx * g.ny + 2 * wl.nb, 9)
    e1 = learned.apply(g, D, ws, r, 0.01)
    e2 = learned.apply(g, D, ws, 2.0 * r, 0.01)
    np.testing.assert_array_equal(e2, 2.0 * e1)
    assert np.linalg.norm(e1) > 0


def _tiny_system():
    from oracle.problem import Problem
    wl = W.tiny(16, 14, 8, 0.3)
    P = Problem(wl, poisson_solver=0)
    g = P.grid
    D = learned.cell_delta(g, wl.xb, wl.yb)
    return wl, P, g, D


def test_energy_loss_bounds_and_optimum():
    # -1 <= loss <= 0 (Cauchy-Schwarz in the K inner product), -1 exactly for
    # a correction parallel to the error, 0 for one K-orthogonal to it
    wl, P, g, D = _tiny_system()
    K = P.ops.K
    rng = np.random.default_rng(3)
    e1 = rng.standard_normal(K.shape[0])
    r1 = K @ e1
    for _ in range(5):
        d = rng.standard_normal(K.shape[0])
        L, _ = learned.energy_loss(d, K @ d, r1, e1)
        assert -1.0 - 1e-12 <= L <= 0.0
    L, gd = learned.energy_loss(-3.0 * e1, K @ (-3.0 * e1), r1, e1)
    assert abs(L + 1.0) < 1e-12 and np.linalg.norm(gd) < 1e-9 * np.linalg.norm(r1)
    d = rng.standard_normal(K.shape[0])
    d -= (d @ (K @ e1)) / (e1 @ (K @ e1)) * e1
    assert abs(learned.energy_loss(d, K @ d, r1, e1)[0]) < 1e-20


def test_energy_loss_gradient_through_the_output_map():
    wl, P, g, D = _tiny_system()
    K = P.ops.K
    rng = np.random.default_rng(4)
    e1 = rng.standard_normal(K.shape[0])
    r1 = K @ e1
    y = rng.standard_normal((3, g.ny, g.nx))
    s, dt = 0.7, wl.dt

    def f(yy):
        d = learned.correction(g, D, yy, s, dt)
        return learned.energy_loss(d, K @ d, r1, e1)

    L, gd = f(y)
    gy = learned.correction_adjoint(g, D, gd, s, dt)
    eps = 1e-6
    for idx in [(0, 2, 3), (1, 7, 8), (2, 6, 9), (0, 13, 15)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += eps
        ym[idx] -= eps
        fd = (f(yp)[0] - f(ym)[0]) / (2 * eps)
        assert abs(fd - gy[idx]) <= 1e-6 * max(1e-3, abs(fd)), (idx, fd, gy[idx])
    # the loss does not change when y is scaled
    assert abs(f(3.5 * y)[0] - L) < 1e-12
