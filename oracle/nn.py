"""FP64 reference of the residual-to-correction network used as a
preconditioner stage (an addition to the paper's method: a small
convolutional network maps the residual left by the AMG V-cycle to a
correction).

Oracle code: test infrastructure only.

Network: L layers of 3x3 convolution, stride 1, zero padding, no bias;
ReLU after every layer except the last.  Tensors are (C, H, W) images;
weights are (C_out, C_in, 3, 3).  The library runs the same network with
BF16 weights and activations and FP32 accumulation; comparisons feed this
oracle the BF16-rounded values, so the only difference left is the
accumulation order and precision.

Convolution (cross-correlation, as in the usual deep-learning definition):
    y[o, i, j] = sum_{c, a, b} W[o, c, a, b] x[c, i + a - 1, j + b - 1]
with x = 0 outside the image.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round FP64/FP32 values to the nearest BF16 (ties to even), returned as FP64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return out.reshape(np.shape(x))


def conv3x3(x, W):
    """Direct definition of the 3x3 zero-padded convolution."""
    C, H, Wd = x.shape
    O = W.shape[0]
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((O, H, Wd))
    for a in range(3):
        for b in range(3):
            patch = xp[:, a:a + H, b:b + Wd]                  # (C, H, W)
            y += np.einsum("oc,chw->ohw", W[:, :, a, b], patch)
    return y


def conv3x3_grad_input(dy, W):
    """dL/dx for y = conv3x3(x, W): the transposed convolution."""
    O, H, Wd = dy.shape
    C = W.shape[1]
    dyp = np.zeros((O, H + 2, Wd + 2))
    dyp[:, 1:-1, 1:-1] = dy
    dx = np.zeros((C, H, Wd))
    for a in range(3):
        for b in range(3):
            # x[c, i+a-1, j+b-1] contributes W[o,c,a,b] dy[o,i,j]
            # => dx[c, p, q] += sum_o W[o,c,a,b] dy[o, p-a+1, q-b+1]
            patch = dyp[:, 2 - a:2 - a + H, 2 - b:2 - b + Wd]
            dx += np.einsum("oc,ohw->chw", W[:, :, a, b], patch)
    return dx


def conv3x3_grad_weight(x, dy):
    """dL/dW for y = conv3x3(x, W)."""
    C, H, Wd = x.shape
    O = dy.shape[0]
    xp = np.zeros((C, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros((O, C, 3, 3))
    for a in range(3):
        for b in range(3):
            dW[:, :, a, b] = np.einsum("ohw,chw->oc", dy, xp[:, a:a + H, b:b + Wd])
    return dW


def forward(weights, x, keep=False):
    """Run the network; returns the output (and the layer inputs if keep)."""
    acts = [x]
    h = x
    for l, W in enumerate(weights):
        h = conv3x3(h, W)
        if l < len(weights) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return (h, acts) if keep else h


def backward(weights, acts, dout):
    """Gradients of a scalar loss with respect to every weight, given dL/dy."""
    grads = [None] * len(weights)
    g = dout
    for l in range(len(weights) - 1, -1, -1):
        if l < len(weights) - 1:
            g = g * (acts[l + 1] > 0.0)          # ReLU mask of this layer's output
        grads[l] = conv3x3_grad_weight(acts[l], g)
        g = conv3x3_grad_input(g, weights[l])
    return grads


def forward_bf16(weights, x, keep=False):
    """The network as the library stores it: input, weights and every hidden
    activation rounded to BF16 (after the ReLU), arithmetic in FP64; the
    output of the last layer is not rounded."""
    wq = [bf16_round(W) for W in weights]
    h = bf16_round(x)
    acts = [h]
    for l, W in enumerate(wq):
        h = conv3x3(h, W)
        if l < len(wq) - 1:
            h = bf16_round(np.maximum(h, 0.0))
        acts.append(h)
    return (h, acts) if keep else h


def backward_bf16(weights, acts, dout):
    """Gradients for forward_bf16: the gradient reaching each layer is masked
    by that layer's ReLU and rounded to BF16 before it meets the BF16
    activations (weight gradient) or the BF16 weights (input gradient)."""
    wq = [bf16_round(W) for W in weights]
    grads = [None] * len(wq)
    g = dout
    for l in range(len(wq) - 1, -1, -1):
        if l < len(wq) - 1:
            g = g * (acts[l + 1] > 0.0)
        g = bf16_round(g)
        grads[l] = conv3x3_grad_weight(acts[l], g)
        g = conv3x3_grad_input(g, wq[l])
    return grads


def nmse_loss(pred, target):
    """Normalised mean squared error sum((p - t)^2) / sum(t^2) and dL/dp."""
    den = float(np.sum(target * target))
    diff = pred - target
    return float(np.sum(diff * diff)) / den, 2.0 * diff / den


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def init_weights(channels, seed):
    """He-normal initialisation for layer shapes channels[l] -> channels[l+1]."""
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        std = np.sqrt(2.0 / (9.0 * cin))
        ws.append(rng.standard_normal((cout, cin, 3, 3)) * std)
    return ws
