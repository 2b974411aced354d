"""Learned warm start: a 4-level U-Net (16-32-64-128 channels, 3x3 convs,
2x2 stride-2 transposed convs for upsampling, 2x2 max pooling) whose every
layer runs in the BF16 MFMA kernels of include/eik_unet.h, trained with the
same kernels (data and weight gradients, Adam). PyTorch only holds the buffers.

Inputs (6 channels, padded to 16): m11, m12, m22, bx, by and the Euclidean
distance d to the nearest source. Output: r = T / (d + h); the warm start is
T_init = r (d + h), so T_init is 0 at the sources.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib as L

CONV3, UP2, DOWN2 = 0, 1, 2

# (name, mode, Cin, Cout, relu) in forward order; the buffers each layer reads
# and writes are wired in UNet._layout.
LAYERS = [
    ("e0a", CONV3, 16, 16, True), ("e0b", CONV3, 16, 16, True),
    ("e1a", CONV3, 16, 32, True), ("e1b", CONV3, 32, 32, True),
    ("e2a", CONV3, 32, 64, True), ("e2b", CONV3, 64, 64, True),
    ("ba", CONV3, 64, 128, True), ("bb", CONV3, 128, 128, True),
    ("u2", UP2, 128, 64, False), ("d2a", CONV3, 128, 64, True), ("d2b", CONV3, 64, 64, True),
    ("u1", UP2, 64, 32, False), ("d1a", CONV3, 64, 32, True), ("d1b", CONV3, 32, 32, True),
    ("u0", UP2, 32, 16, False), ("d0a", CONV3, 32, 16, True), ("d0b", CONV3, 16, 16, True),
]


def _bind():
    lib = L.lib()
    if getattr(lib, "_eiku_bound", False):
        return lib
    i32, i64, vp, f = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_float
    sig = {
        "eiku_conv_fwd": [i32, i32, i32, i32, vp, i32, i32, i32, vp, vp, i32, vp, i32, i32, i32, vp],
        "eiku_conv_wgrad": [i32, i32, i32, i32, vp, i32, i32, i32, vp, i32, i32, i32, vp, vp],
        "eiku_conv_fwd_cat": [i32, i32, i32, vp, i32, i32, i32, vp, i32, i32, i32, vp, vp, i32, vp, i32, i32, i32, vp],
        "eiku_conv_wgrad_cat": [i32, i32, i32, vp, i32, i32, i32, vp, i32, i32, i32, vp, i32, i32, i32, vp, vp],
        "eiku_bias_grad": [i64, vp, i32, i32, i32, vp, vp],
        "eiku_relu_mask": [i64, vp, i32, i32, vp, i32, i32, i32, vp],
        "eiku_add": [i64, vp, i32, i32, vp, i32, i32, i32, vp],
        "eiku_maxpool_fwd": [i32, i32, i32, vp, i32, i32, vp, i32, i32, i32, vp],
        "eiku_maxpool_bwd": [i32, i32, i32, vp, i32, i32, vp, i32, i32, vp, i32, i32, i32, vp],
        "eiku_head_fwd": [i64, vp, i32, i32, i32, vp, vp, vp, vp],
        "eiku_head_bwd": [i64, vp, i32, i32, i32, vp, vp, vp, i32, i32, vp, vp, vp],
        "eiku_features": [i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp],
        "eiku_mse": [i64, vp, vp, vp, vp, vp],
        "eiku_adam": [i64, vp, vp, vp, vp, f, f, f, f, i32, vp],
        "eiku_prep_weights": [i32, i32, i32, i32, i32, vp, vp, vp, vp],
        "eiku_to_bf16": [i64, vp, vp, vp],
        "eiku_to_f32": [i64, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib._eiku_bound = True
    return lib


def _ok(name, rc):
    if rc != 0:
        raise RuntimeError(f"{name} rejected its arguments")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Act:
    """A view into an NHWC bf16 buffer: (tensor, grid, channel stride, offset, channels)."""

    def __init__(self, buf, B, H, W, cs, co, C):
        self.buf, self.B, self.H, self.W, self.cs, self.co, self.C = buf, B, H, W, cs, co, C

    @property
    def npix(self):
        return self.B * self.H * self.W


class Cat:
    """The concatenation [a | b] of two views on the same grid, read from the
    two producers' own buffers (each producer writes whole pixels)."""

    def __init__(self, a, b):
        assert (a.B, a.H, a.W) == (b.B, b.H, b.W)
        self.a, self.b = a, b
        self.B, self.H, self.W, self.C = a.B, a.H, a.W, a.C + b.C

    @property
    def npix(self):
        return self.B * self.H * self.W


# skip and upsampled halves of each level's concatenation; their gradients
# share one buffer per level (the data gradient of the next convolution
# writes both halves of every pixel at once)
SPLIT = {"s0": ("g_cat0", 0), "up0": ("g_cat0", 1), "s1": ("g_cat1", 0), "up1": ("g_cat1", 1), "s2": ("g_cat2", 0),
         "up2": ("g_cat2", 1)}


class UNet:
    def __init__(self, device="cuda", seed=0):
        self.dev = torch.device(device)
        self.lib = _bind()
        g = torch.Generator().manual_seed(seed)
        self.params = {}
        for name, mode, cin, cout, _ in LAYERS:
            taps = 9 if mode == CONV3 else 4
            fan_in = taps * (6 if name == "e0a" else cin)
            w = torch.randn(taps, cout, cin, generator=g) * math.sqrt(2.0 / fan_in)
            if name == "e0a":
                w[:, :, 6:] = 0.0  # input channels beyond the six features are zero padding
            self.params[name + ".w"] = w
            self.params[name + ".b"] = torch.zeros(cout)
        self.params["head.w"] = torch.randn(16, generator=g) * math.sqrt(1.0 / 16)
        self.params["head.b"] = torch.ones(1)
        self.params = {k: v.to(self.dev, torch.float32).contiguous() for k, v in self.params.items()}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.step_count = 0
        self.wf, self.wb = {}, {}
        self._bufs = None
        self.refresh_weights()

    # -- weights ----------------------------------------------------------
    def refresh_weights(self):
        st = L.stream_handle(self.dev)
        for name, mode, cin, cout, _ in LAYERS:
            taps = 9 if mode == CONV3 else 4
            w = self.params[name + ".w"]
            if name not in self.wf:
                self.wf[name] = torch.empty(taps, cout, cin, dtype=torch.int16, device=self.dev)
                self.wb[name] = torch.empty(taps, cin, cout, dtype=torch.int16, device=self.dev)
            _ok("eiku_prep_weights", self.lib.eiku_prep_weights(mode, taps, cout, cin, cin, _p(w), _p(self.wf[name]),
                                                                _p(self.wb[name]), st))

    def state_dict(self):
        return {k: v.detach().cpu() for k, v in self.params.items()}

    def load_state_dict(self, sd):
        for k, v in sd.items():
            self.params[k].copy_(v.to(self.dev, torch.float32))
        self.refresh_weights()

    # -- buffers ----------------------------------------------------------
    def _layout(self, B, H, W):
        if self._bufs is not None and self._bufs["shape"] == (B, H, W):
            return self._bufs
        assert H % 8 == 0 and W % 8 == 0, "grid sides must be multiples of 8 (three 2x2 poolings)"
        d = self.dev

        def buf(h, w, c):
            return torch.zeros(B * h * w * c, dtype=torch.int16, device=d)

        H1, W1, H2, W2, H3, W3 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8
        b = {"shape": (B, H, W)}
        b["x0"] = buf(H, W, 16)
        for k, (h, w, c) in {"e0a": (H, W, 16), "s0": (H, W, 16), "up0": (H, W, 16), "d0a": (H, W, 16),
                             "d0b": (H, W, 16), "p0": (H1, W1, 16), "e1a": (H1, W1, 32), "s1": (H1, W1, 32),
                             "up1": (H1, W1, 32), "d1a": (H1, W1, 32), "d1b": (H1, W1, 32), "p1": (H2, W2, 32),
                             "e2a": (H2, W2, 64), "s2": (H2, W2, 64), "up2": (H2, W2, 64), "d2a": (H2, W2, 64),
                             "d2b": (H2, W2, 64), "p2": (H3, W3, 64), "ba": (H3, W3, 128), "bb": (H3, W3, 128)}.items():
            b[k] = buf(h, w, c)
            if k not in SPLIT:
                b["g_" + k] = buf(h, w, c)
        for lv, (h, w, c) in enumerate([(H, W, 16), (H1, W1, 32), (H2, W2, 64)]):
            b[f"g_cat{lv}"] = buf(h, w, 2 * c)
        b["g_pool"] = buf(H, W, 16)  # scratch for max-pool gradients (largest level)
        b["pred"] = torch.zeros(B * H * W, dtype=torch.float32, device=d)
        b["g_pred"] = torch.zeros(B * H * W, dtype=torch.float32, device=d)
        b["g_x0"] = buf(H, W, 16)
        self._bufs = b
        return b

    def _wiring(self, b, B, H, W):
        """(input Act, output Act) of every layer."""
        H1, W1, H2, W2, H3, W3 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8

        def A(k, h, w, cs, co, c):
            return Act(b[k], B, h, w, cs, co, c)

        return {
            "e0a": (A("x0", H, W, 16, 0, 16), A("e0a", H, W, 16, 0, 16)),
            "e0b": (A("e0a", H, W, 16, 0, 16), A("s0", H, W, 16, 0, 16)),
            "e1a": (A("p0", H1, W1, 16, 0, 16), A("e1a", H1, W1, 32, 0, 32)),
            "e1b": (A("e1a", H1, W1, 32, 0, 32), A("s1", H1, W1, 32, 0, 32)),
            "e2a": (A("p1", H2, W2, 32, 0, 32), A("e2a", H2, W2, 64, 0, 64)),
            "e2b": (A("e2a", H2, W2, 64, 0, 64), A("s2", H2, W2, 64, 0, 64)),
            "ba": (A("p2", H3, W3, 64, 0, 64), A("ba", H3, W3, 128, 0, 128)),
            "bb": (A("ba", H3, W3, 128, 0, 128), A("bb", H3, W3, 128, 0, 128)),
            "u2": (A("bb", H3, W3, 128, 0, 128), A("up2", H2, W2, 64, 0, 64)),
            "d2a": (Cat(A("s2", H2, W2, 64, 0, 64), A("up2", H2, W2, 64, 0, 64)), A("d2a", H2, W2, 64, 0, 64)),
            "d2b": (A("d2a", H2, W2, 64, 0, 64), A("d2b", H2, W2, 64, 0, 64)),
            "u1": (A("d2b", H2, W2, 64, 0, 64), A("up1", H1, W1, 32, 0, 32)),
            "d1a": (Cat(A("s1", H1, W1, 32, 0, 32), A("up1", H1, W1, 32, 0, 32)), A("d1a", H1, W1, 32, 0, 32)),
            "d1b": (A("d1a", H1, W1, 32, 0, 32), A("d1b", H1, W1, 32, 0, 32)),
            "u0": (A("d1b", H1, W1, 32, 0, 32), A("up0", H, W, 16, 0, 16)),
            "d0a": (Cat(A("s0", H, W, 16, 0, 16), A("up0", H, W, 16, 0, 16)), A("d0a", H, W, 16, 0, 16)),
            "d0b": (A("d0a", H, W, 16, 0, 16), A("d0b", H, W, 16, 0, 16)),
        }

    # -- forward ----------------------------------------------------------
    def features(self, M, omega, src, h):
        """M (B,3,H,W), omega (B,2,H,W) float32; src (B, max_src) int32 (-1 unused);
        h (B,) float32. Fills the input buffer; returns d (B,H,W)."""
        B, _, H, W = M.shape
        b = self._layout(B, H, W)
        dist = torch.empty(B, H, W, dtype=torch.float32, device=self.dev)
        _ok("eiku_features", self.lib.eiku_features(B, H, W, _p(M), _p(omega), _p(src), src.shape[1], _p(h),
                                                    _p(b["x0"]), _p(dist), L.stream_handle(self.dev)))
        return dist

    def _conv(self, name, mode, x, y, relu):
        st = L.stream_handle(self.dev)
        B, H, W = (x.B, x.H, x.W)
        if isinstance(x, Cat):
            assert mode == CONV3
            xa, xb = x.a, x.b
            _ok(name, self.lib.eiku_conv_fwd_cat(B, H, W, _p(xa.buf), xa.cs, xa.co, xa.C, _p(xb.buf), xb.cs, xb.co,
                                                 xb.C, _p(self.wf[name]), _p(self.params[name + ".b"]), int(relu),
                                                 _p(y.buf), y.cs, y.co, y.C, st))
            return
        _ok(name, self.lib.eiku_conv_fwd(mode, B, H, W, _p(x.buf), x.cs, x.co, x.C, _p(self.wf[name]),
                                         _p(self.params[name + ".b"]), int(relu), _p(y.buf), y.cs, y.co, y.C, st))

    def forward(self, B, H, W):
        """Runs the network on the input buffer; returns the prediction (B*H*W) float32."""
        b = self._layout(B, H, W)
        wire = self._wiring(b, B, H, W)
        st = L.stream_handle(self.dev)
        H1, W1, H2, W2, H3, W3 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8
        for name, mode, cin, cout, relu in LAYERS:
            x, y = wire[name]
            self._conv(name, mode, x, y, relu)
            if name == "e0b":
                _ok("pool0", self.lib.eiku_maxpool_fwd(B, H1, W1, _p(b["s0"]), 16, 0, _p(b["p0"]), 16, 0, 16, st))
            elif name == "e1b":
                _ok("pool1", self.lib.eiku_maxpool_fwd(B, H2, W2, _p(b["s1"]), 32, 0, _p(b["p1"]), 32, 0, 32, st))
            elif name == "e2b":
                _ok("pool2", self.lib.eiku_maxpool_fwd(B, H3, W3, _p(b["s2"]), 64, 0, _p(b["p2"]), 64, 0, 64, st))
        _ok("head", self.lib.eiku_head_fwd(B * H * W, _p(b["d0b"]), 16, 0, 16, _p(self.params["head.w"]),
                                           _p(self.params["head.b"]), _p(b["pred"]), st))
        return b["pred"]

    # -- backward ---------------------------------------------------------
    def backward(self, B, H, W):
        """Back-propagates g_pred (already in the buffer) into self.grads."""
        b = self._layout(B, H, W)
        wire = self._wiring(b, B, H, W)
        st = L.stream_handle(self.dev)
        lib = self.lib
        H1, W1, H2, W2, H3, W3 = H // 2, W // 2, H // 4, W // 4, H // 8, W // 8
        n0 = B * H * W
        _ok("head_bwd", lib.eiku_head_bwd(n0, _p(b["d0b"]), 16, 0, 16, _p(self.params["head.w"]), _p(b["g_pred"]),
                                          _p(b["g_d0b"]), 16, 0, _p(self.grads["head.w"]), _p(self.grads["head.b"]),
                                          st))
        def key_of(a):
            return [k for k, v in b.items() if v is a.buf][0]

        def gof(a):  # gradient view matching an activation view
            if isinstance(a, Cat):  # both halves: the level's whole gradient buffer
                return Act(b[SPLIT[key_of(a.a)][0]], a.B, a.H, a.W, a.C, 0, a.C)
            key = key_of(a)
            if key in SPLIT:
                g, half = SPLIT[key]
                return Act(b[g], a.B, a.H, a.W, 2 * a.C, half * a.C, a.C)
            return Act(b["g_" + key], a.B, a.H, a.W, a.cs, a.co, a.C)

        # layer whose input came from max pooling of a skip tensor: (skip, pooled, channels, pooled grid)
        pools = {"e1a": ("s0", "p0", 16, H1, W1), "e2a": ("s1", "p1", 32, H2, W2), "ba": ("s2", "p2", 64, H3, W3)}
        for name, mode, cin, cout, relu in reversed(LAYERS):
            x, y = wire[name]
            gy, gx = gof(y), gof(x)
            if relu:
                _ok("relu_mask", lib.eiku_relu_mask(y.npix, _p(y.buf), y.cs, y.co, _p(gy.buf), gy.cs, gy.co, y.C, st))
            if isinstance(x, Cat):
                xa, xb = x.a, x.b
                _ok("wgrad", lib.eiku_conv_wgrad_cat(y.B, y.H, y.W, _p(xa.buf), xa.cs, xa.co, xa.C, _p(xb.buf), xb.cs,
                                                     xb.co, xb.C, _p(gy.buf), gy.cs, gy.co, y.C,
                                                     _p(self.grads[name + ".w"]), st))
            elif mode == CONV3:
                _ok("wgrad", lib.eiku_conv_wgrad(CONV3, y.B, y.H, y.W, _p(x.buf), x.cs, x.co, x.C, _p(gy.buf), gy.cs,
                                                 gy.co, y.C, _p(self.grads[name + ".w"]), st))
            else:
                _ok("wgrad", lib.eiku_conv_wgrad(UP2, x.B, x.H, x.W, _p(x.buf), x.cs, x.co, x.C, _p(gy.buf), gy.cs,
                                                 gy.co, y.C, _p(self.grads[name + ".w"]), st))
            _ok("bias_grad", lib.eiku_bias_grad(y.npix, _p(gy.buf), gy.cs, gy.co, y.C, _p(self.grads[name + ".b"]),
                                                st))
            if name == "e0a":
                continue  # no gradient for the inputs
            if mode == CONV3:
                _ok("dgrad", lib.eiku_conv_fwd(CONV3, x.B, x.H, x.W, _p(gy.buf), gy.cs, gy.co, y.C, _p(self.wb[name]),
                                               None, 0, _p(gx.buf), gx.cs, gx.co, x.C, st))
            else:
                _ok("dgrad", lib.eiku_conv_fwd(DOWN2, x.B, x.H, x.W, _p(gy.buf), gy.cs, gy.co, y.C,
                                               _p(self.wb[name]), None, 0, _p(gx.buf), gx.cs, gx.co, x.C, st))
            if name in pools:  # the input came from max pooling of a skip tensor: route and add
                src, pk, C, hp, wp = pools[name]
                gs = gof(Act(b[src], B, 2 * hp, 2 * wp, C, 0, C))
                _ok("pool_bwd", lib.eiku_maxpool_bwd(B, hp, wp, _p(b[src]), C, 0, _p(b["g_" + pk]), C, 0,
                                                     _p(b["g_pool"]), C, 0, C, st))
                _ok("add", lib.eiku_add(B * hp * 2 * wp * 2, _p(gs.buf), gs.cs, gs.co, _p(b["g_pool"]), C, 0, C, st))

    # -- optimiser ----------------------------------------------------------
    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        st = L.stream_handle(self.dev)
        for k in self.params:
            p = self.params[k]
            _ok("adam", self.lib.eiku_adam(p.numel(), _p(p), _p(self.grads[k]), _p(self.m[k]), _p(self.v[k]), lr,
                                           beta1, beta2, eps, self.step_count, st))
        self.refresh_weights()

    def zero_grads(self):
        for g in self.grads.values():
            g.zero_()

    def train_step(self, target, lr=1e-3):
        """target: (B*H*W) float32 on the device; inputs already in the buffer."""
        B, H, W = self._bufs["shape"]
        pred = self.forward(B, H, W)
        loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        _ok("mse", self.lib.eiku_mse(pred.numel(), _p(pred), _p(target), _p(loss), _p(self._bufs["g_pred"]),
                                     L.stream_handle(self.dev)))
        self.backward(B, H, W)
        self.adam_step(lr)
        return loss
