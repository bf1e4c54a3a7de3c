"""Pins of the FP64 network oracle: the convolution against scipy's
correlate2d, gradients against central finite differences, and the
BF16 rounding against exactly representable values."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 9, 11))
    W = rng.standard_normal((4, 3, 3, 3))
    y = nn.conv3x3(x, W)
    for o in range(4):
        ref = sum(correlate2d(x[c], W[o, c], mode="same", boundary="fill") for c in range(3))
        np.testing.assert_allclose(y[o], ref, rtol=1e-13, atol=1e-13)


def test_conv_identity_and_shift_kernels():
    x = np.random.default_rng(1).standard_normal((1, 6, 7))
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 1, 1] = 1.0
    np.testing.assert_array_equal(nn.conv3x3(x, W), x)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 1, 2] = 1.0                     # y[i, j] = x[i, j+1]
    y = nn.conv3x3(x, W)
    np.testing.assert_array_equal(y[0, :, :-1], x[0, :, 1:])
    assert np.all(y[0, :, -1] == 0.0)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    ws = nn.init_weights([2, 4, 4, 2], seed=3)
    x = rng.standard_normal((2, 7, 6))
    t = rng.standard_normal((2, 7, 6))
    out, acts = nn.forward(ws, x, keep=True)
    loss, dout = nn.nmse_loss(out, t)
    grads = nn.backward(ws, acts, dout)
    eps = 1e-6
    for l in range(len(ws)):
        for idx in [(0, 0, 0, 0), (1, 1, 2, 1), (ws[l].shape[0] - 1, ws[l].shape[1] - 1, 1, 2)]:
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += eps
            wm[l][idx] -= eps
            fd = (nn.nmse_loss(nn.forward(wp, x), t)[0] - nn.nmse_loss(nn.forward(wm, x), t)[0]) / (2 * eps)
            assert abs(fd - grads[l][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][idx])
    # input gradient of a single linear layer against finite differences
    W = rng.standard_normal((3, 2, 3, 3))
    dy = rng.standard_normal((3, 7, 6))
    dx = nn.conv3x3_grad_input(dy, W)
    for idx in [(0, 0, 0), (1, 3, 2), (1, 6, 5)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (np.sum(nn.conv3x3(xp, W) * dy) - np.sum(nn.conv3x3(xm, W) * dy)) / (2 * eps)
        assert abs(fd - dx[idx]) <= 1e-7 * max(1.0, abs(fd))


def test_bf16_rounding():
    vals = np.array([1.0, -2.0, 0.5, 3.140625, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65280.0])
    r = nn.bf16_round(vals)
    # exactly representable values stay; ties round to even
    assert r[0] == 1.0 and r[1] == -2.0 and r[2] == 0.5 and r[3] == 3.140625
    assert r[4] == 1.0                       # 1 + 2^-8 is a tie -> even (1.0)
    assert r[5] == 1.0 + 2.0 ** -6           # 1 + 3*2^-8 is a tie -> even (1 + 4*2^-8)
    x = np.random.default_rng(4).standard_normal(1000)
    rel = np.abs(nn.bf16_round(x) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -8 + 1e-12


def test_adam_first_step_moves_by_lr():
    w = np.array([1.0, -1.0])
    g = np.array([0.3, -5.0])
    w1, m, v = nn.adam_step(w, g, np.zeros(2), np.zeros(2), 1, lr=0.01)
    np.testing.assert_allclose(w1, w - 0.01 * np.sign(g), rtol=0, atol=1e-9)
