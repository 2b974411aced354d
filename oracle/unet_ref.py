"""Oracle for the warm-start network's layers: plain float64 numpy on
bfloat16-rounded operands.

TEST INFRASTRUCTURE (see oracle/__init__.py). Tensors are NHWC (B, H, W, C);
3x3 weights are (9, Cout, Cin) with tap t at offset (t // 3 - 1, t % 3 - 1) in
(y, x); 2x2 stride-2 transposed-convolution weights are (4, Cout, Cin) with tap
2 a + c writing output pixel (2 y + a, 2 x + c). Each function is the
definition of the layer written out over its taps.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    u = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def from_bits(b):
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


def conv3(x, w, bias=None, relu=False):
    B, H, W, _ = x.shape
    xp = np.zeros((B, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.zeros((B, H, W, w.shape[1]))
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        y += xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W] @ w[t].T
    if bias is not None:
        y += bias
    return np.maximum(y, 0.0) if relu else y


def conv3_wgrad(x, dy):
    """dW[t, co, ci] = sum over pixels of dy(p, co) x(p + d_t, ci)."""
    B, H, W, _ = x.shape
    xp = np.zeros((B, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1] = x
    out = np.zeros((9, dy.shape[3], x.shape[3]))
    for t in range(9):
        ddy, ddx = t // 3 - 1, t % 3 - 1
        xs = xp[:, 1 + ddy:1 + ddy + H, 1 + ddx:1 + ddx + W].reshape(-1, x.shape[3])
        out[t] = dy.reshape(-1, dy.shape[3]).T @ xs
    return out


def up2(x, w, bias=None):
    B, H, W, _ = x.shape
    y = np.zeros((B, 2 * H, 2 * W, w.shape[1]))
    for t in range(4):
        a, c = t >> 1, t & 1
        y[:, a::2, c::2] = x @ w[t].T
    if bias is not None:
        y += bias
    return y


def down2(x, w):
    """Data gradient of up2: y(p) = sum_{a, c} x(2y + a, 2x + c) W[2a + c]."""
    B, H2, W2, _ = x.shape
    y = np.zeros((B, H2 // 2, W2 // 2, w.shape[1]))
    for t in range(4):
        a, c = t >> 1, t & 1
        y += x[:, a::2, c::2] @ w[t].T
    return y


def up2_wgrad(x, dy):
    out = np.zeros((4, dy.shape[3], x.shape[3]))
    for t in range(4):
        a, c = t >> 1, t & 1
        out[t] = dy[:, a::2, c::2].reshape(-1, dy.shape[3]).T @ x.reshape(-1, x.shape[3])
    return out


def maxpool(x):
    B, H2, W2, C = x.shape
    return x.reshape(B, H2 // 2, 2, W2 // 2, 2, C).max(axis=(2, 4))


def maxpool_bwd(x, dy):
    """The first maximum of each 2x2 window (order (0,0), (0,1), (1,0), (1,1)) gets dy."""
    B, H2, W2, C = x.shape
    win = x.reshape(B, H2 // 2, 2, W2 // 2, 2, C).transpose(0, 1, 3, 5, 2, 4).reshape(B, H2 // 2, W2 // 2, C, 4)
    arg = win.argmax(axis=-1)
    dx = np.zeros_like(x)
    for q in range(4):
        a, c = q >> 1, q & 1
        dx[:, a::2, c::2] = np.where(arg == q, dy, 0.0)
    return dx


def head(x, w, b):
    return x @ w + b
