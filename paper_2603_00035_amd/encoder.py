"""Covariate encoder trained end to end through the solver (Sec. 6, encoder
architecture and learning framework; App. wildfire experiments, training
protocol), on synthetic covariates.

Two pathways, as in the paper: a fully convolutional network over the spatial
covariates Y(x) (four 3x3 convolutions with ReLU, 16 -> 64 -> 64 -> 64 -> 16
channels, then five 1x1 heads giving G_local and b_local: 5 layers with 64
hidden channels, about 93 K parameters) and a
dense network over the global covariates y (one hidden layer of 32 with ReLU)
giving the baseline (G0, b0); combined as G = G0 + alpha G_local,
b = b0 + alpha b_local and projected onto the feasible set. Training takes
the hybrid gradient: the data term's gradient with respect to (G, b) from the
implicit adjoint (eik_backward), then back through the projection, the
combination and both pathways; the TV regulariser on (G, b) is added to that
gradient directly.

Every step is a library call: the convolutions, ReLU masks, heads, data and
weight gradients and Adam are the BF16 MFMA kernels of eik_unet.h; the dense
layers and the combination are eik_encoder.h; projection, solve, data term,
adjoint and TV are eik.h / eik_inverse.h. PyTorch only holds the buffers and
lays the covariates out once per scene (NHWC, padded to 16 channels).
Several scenes of one size train together (Trainer.step_batch): the network
runs on the batch, the solves and adjoints are one batched launch, and the
projection runs per scene.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib as L
from . import eikonal as E
from . import inverse as I
from .unet import CONV3, _bind, _ok, _p

CONV_LAYERS = [("c1", 16, 64), ("c2", 64, 64), ("c3", 64, 64), ("c4", 64, 16)]
HEAD_IN = CONV_LAYERS[-1][2]  # channels the 1x1 heads read
CONV_NAMES = [c[0] for c in CONV_LAYERS]
N_HEADS = 5          # g11, g12, g22, b1, b2
HIDDEN = 32
BASE_INIT = (1.0, 0.0, 1.0, 0.0, 0.0)


class Encoder:
    def __init__(self, n_cov=4, n_global=4, alpha=0.5, device="cuda", seed=0):
        if not 1 <= n_cov <= 16:
            raise ValueError("1..16 spatial covariates")
        self.dev = torch.device(device)
        self.lib = _bind()
        self.n_cov, self.n_global, self.alpha = n_cov, n_global, float(alpha)
        g = torch.Generator().manual_seed(seed)
        p = {}
        for name, cin, cout in CONV_LAYERS:
            fan_in = 9 * (n_cov if name == "c1" else cin)
            w = torch.randn(9, cout, cin, generator=g) * math.sqrt(2.0 / fan_in)
            if name == "c1":
                w[:, :, n_cov:] = 0.0
            p[name + ".w"], p[name + ".b"] = w, torch.zeros(cout)
        for k in range(N_HEADS):
            p[f"head{k}.w"] = torch.randn(HEAD_IN, generator=g) * (0.05 / math.sqrt(HEAD_IN))
            p[f"head{k}.b"] = torch.zeros(1)
        p["g1.w"] = torch.randn(HIDDEN, n_global, generator=g) * math.sqrt(2.0 / n_global)
        p["g1.b"] = torch.zeros(HIDDEN)
        p["g2.w"] = torch.randn(N_HEADS, HIDDEN, generator=g) * 0.01
        p["g2.b"] = torch.tensor(BASE_INIT)
        self.params = {k: v.to(self.dev, torch.float32).contiguous() for k, v in p.items()}
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.t = 0
        self.wf, self.wb = {}, {}
        self.shape = None
        self.refresh_weights()

    def n_params(self):
        return sum(v.numel() for v in self.params.values())

    def refresh_weights(self):
        st = L.stream_handle(self.dev)
        for name, cin, cout in CONV_LAYERS:
            if name not in self.wf:
                self.wf[name] = torch.empty(9, cout, cin, dtype=torch.int16, device=self.dev)
                self.wb[name] = torch.empty(9, cin, cout, dtype=torch.int16, device=self.dev)
            _ok("eiku_prep_weights", self.lib.eiku_prep_weights(CONV3, 9, cout, cin, cin, _p(self.params[name + ".w"]),
                                                                _p(self.wf[name]), _p(self.wb[name]), st))

    def state_dict(self):
        return {k: v.detach().cpu().clone() for k, v in self.params.items()}

    # -- buffers ----------------------------------------------------------
    def _alloc(self, B, H, W):
        if self.shape == (B, H, W):
            return
        n, d = B * H * W, self.dev
        self.shape = (B, H, W)
        self.x0 = torch.zeros(n * 16, dtype=torch.int16, device=d)
        self.act = {name: torch.zeros(n * cout, dtype=torch.int16, device=d) for name, _, cout in CONV_LAYERS}
        self.gact = {name: torch.zeros(n * cout, dtype=torch.int16, device=d) for name, _, cout in CONV_LAYERS}
        self.gtmp = torch.zeros(n * HEAD_IN, dtype=torch.int16, device=d)
        self.local = torch.zeros(N_HEADS, B, H, W, dtype=torch.float32, device=d)
        self.dlocal = torch.zeros(N_HEADS, B, H, W, dtype=torch.float32, device=d)
        self.yg = torch.zeros(B, self.n_global, dtype=torch.float32, device=d)
        self.hid = torch.zeros(B, HIDDEN, dtype=torch.float32, device=d)
        self.dhid = torch.zeros(B, HIDDEN, dtype=torch.float32, device=d)
        self.base = torch.zeros(B, N_HEADS, dtype=torch.float32, device=d)
        self.dbase = torch.zeros(B, N_HEADS, dtype=torch.float32, device=d)
        self.scratch = torch.empty(L.lib().eik_enc_scratch_bytes(B), dtype=torch.uint8, device=d)

    def set_inputs(self, X, y):
        """X (n_cov, H, W) and y (n_global,) for one scene, or X (B, n_cov,
        H, W) and y (B, n_global) for a batch of B scenes of one size."""
        self.batched = X.dim() == 4
        X = X if self.batched else X.unsqueeze(0)
        B, _, H, W = X.shape
        self._alloc(B, H, W)
        Xp = torch.zeros(B, H, W, 16, dtype=torch.float32, device=self.dev)
        Xp[..., :self.n_cov] = X.to(self.dev, torch.float32).permute(0, 2, 3, 1)
        _ok("eiku_to_bf16", self.lib.eiku_to_bf16(Xp.numel(), _p(Xp), _p(self.x0), L.stream_handle(self.dev)))
        self.yg.copy_(y.to(self.dev, torch.float32).view(B, -1))

    # -- forward ----------------------------------------------------------
    def forward(self, dtype=torch.float32):
        """(M, omega) before the projection: (3, H, W) and (2, H, W) for one
        scene, (B, 3, H, W) and (B, 2, H, W) for a batch."""
        B, H, W = self.shape
        n = H * W
        st = L.stream_handle(self.dev)
        lib, enc = self.lib, L.lib()
        x, cx = self.x0, 16
        for name, cin, cout in CONV_LAYERS:
            _ok(name, lib.eiku_conv_fwd(CONV3, B, H, W, _p(x), cx, 0, cin, _p(self.wf[name]),
                                        _p(self.params[name + ".b"]), 1, _p(self.act[name]), cout, 0, cout, st))
            x, cx = self.act[name], cout
        for k in range(N_HEADS):
            _ok("head", lib.eiku_head_fwd(B * n, _p(x), HEAD_IN, 0, HEAD_IN, _p(self.params[f"head{k}.w"]),
                                          _p(self.params[f"head{k}.b"]), _p(self.local[k]), st))
        L.check("eik_enc_dense", enc.eik_enc_dense(B, self.n_global, HIDDEN, L.ptr(self.yg), L.ptr(self.params["g1.w"]),
                                                   L.ptr(self.params["g1.b"]), 1, L.ptr(self.hid), st))
        L.check("eik_enc_dense", enc.eik_enc_dense(B, HIDDEN, N_HEADS, L.ptr(self.hid), L.ptr(self.params["g2.w"]),
                                                   L.ptr(self.params["g2.b"]), 0, L.ptr(self.base), st))
        M = torch.empty(B, 3, H, W, dtype=dtype, device=self.dev)
        om = torch.empty(B, 2, H, W, dtype=dtype, device=self.dev)
        L.check("eik_enc_combine", enc.eik_enc_combine(B, n, L.dtype_code(M), self.alpha, L.ptr(self.base),
                                                       L.ptr(self.local), L.ptr(M), L.ptr(om), st))
        return (M, om) if self.batched else (M[0], om[0])

    # -- backward ---------------------------------------------------------
    def backward(self, dM, dom):
        """Accumulates into self.grads the gradients of sum(dM * M) +
        sum(dom * omega) for the last forward's (M, omega)."""
        B, H, W = self.shape
        n = H * W
        npix = B * n
        st = L.stream_handle(self.dev)
        lib, enc = self.lib, L.lib()
        self.dbase.zero_()
        dM, dom = dM.contiguous(), dom.contiguous()
        if dM.numel() != B * 3 * n or dom.numel() != B * 2 * n:
            raise ValueError("gradients must match the last forward's (M, omega)")
        L.check("eik_enc_combine_backward",
                enc.eik_enc_combine_backward(B, n, L.dtype_code(dM), self.alpha, L.ptr(dM), L.ptr(dom),
                                             L.ptr(self.dlocal), L.ptr(self.dbase), L.ptr(self.scratch), st))
        L.check("eik_enc_dense_backward",
                enc.eik_enc_dense_backward(B, HIDDEN, N_HEADS, L.ptr(self.hid), L.ptr(self.params["g2.w"]),
                                           L.ptr(self.base), 0, L.ptr(self.dbase), L.ptr(self.dhid),
                                           L.ptr(self.grads["g2.w"]), L.ptr(self.grads["g2.b"]), st))
        L.check("eik_enc_dense_backward",
                enc.eik_enc_dense_backward(B, self.n_global, HIDDEN, L.ptr(self.yg), L.ptr(self.params["g1.w"]),
                                           L.ptr(self.hid), 1, L.ptr(self.dhid), None, L.ptr(self.grads["g1.w"]),
                                           L.ptr(self.grads["g1.b"]), st))
        top = CONV_NAMES[-1]
        for k in range(N_HEADS):
            dst = self.gact[top] if k == 0 else self.gtmp
            _ok("head_bwd", lib.eiku_head_bwd(npix, _p(self.act[top]), HEAD_IN, 0, HEAD_IN,
                                              _p(self.params[f"head{k}.w"]), _p(self.dlocal[k]), _p(dst), HEAD_IN, 0,
                                              _p(self.grads[f"head{k}.w"]), _p(self.grads[f"head{k}.b"]), st))
            if k > 0:
                _ok("add", lib.eiku_add(npix, _p(self.gact[top]), HEAD_IN, 0, _p(self.gtmp), HEAD_IN, 0, HEAD_IN, st))
        for li in range(len(CONV_LAYERS) - 1, -1, -1):
            name, cin, cout = CONV_LAYERS[li]
            y, gy = self.act[name], self.gact[name]
            x, cx = (self.x0, 16) if li == 0 else (self.act[CONV_NAMES[li - 1]], cin)
            _ok("relu_mask", lib.eiku_relu_mask(npix, _p(y), cout, 0, _p(gy), cout, 0, cout, st))
            _ok("wgrad", lib.eiku_conv_wgrad(CONV3, B, H, W, _p(x), cx, 0, cin, _p(gy), cout, 0, cout,
                                             _p(self.grads[name + ".w"]), st))
            _ok("bias_grad", lib.eiku_bias_grad(npix, _p(gy), cout, 0, cout, _p(self.grads[name + ".b"]), st))
            if li > 0:
                gx = self.gact[CONV_NAMES[li - 1]]
                _ok("dgrad", lib.eiku_conv_fwd(CONV3, B, H, W, _p(gy), cout, 0, cout, _p(self.wb[name]), None, 0,
                                               _p(gx), cin, 0, cin, st))

    def zero_grads(self):
        for g in self.grads.values():
            g.zero_()

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """Adam on every parameter (clears the gradients), then the BF16
        copies of the convolution weights."""
        self.t += 1
        st = L.stream_handle(self.dev)
        for k, p in self.params.items():
            _ok("adam", self.lib.eiku_adam(p.numel(), _p(p), _p(self.grads[k]), _p(self.m[k]), _p(self.v[k]), lr,
                                           beta1, beta2, eps, self.t, st))
        self.refresh_weights()


class Trainer:
    """Hybrid training on scenes (covariates, ignition, observed arrival
    times with a mask of observed nodes)."""

    def __init__(self, enc: Encoder, lam_tv=0.0, tol=1e-5, lr=1e-3):
        self.enc, self.lam_tv, self.tol, self.lr = enc, float(lam_tv), float(tol), float(lr)
        self.scratch = torch.empty(L.lib().eik_inv_scratch_bytes(), dtype=torch.uint8, device=enc.dev)
        self.scalars = torch.zeros(3, dtype=torch.float64, device=enc.dev)

    def predict(self, X, y, src, h, src_t=None):
        self.enc.set_inputs(X, y)
        M, om = self.enc.forward()
        Mp, op = E.project(M, om)
        T, par, _, _ = E.solve(Mp, op, src, h, src_t=src_t, tol=self.tol, levels=False)
        return T, (M, om, Mp, op, par)

    def gradients(self, X, y, src, h, T_obs, mask, src_t=None):
        """Forward, data term, implicit adjoint, projection VJP and encoder
        backward; accumulates into enc.grads. Returns (T, device scalars
        (data term, lam R(G), lam R(b)))."""
        T, (M, om, Mp, op, par) = self.predict(X, y, src, h, src_t)
        st = L.stream_handle(self.enc.dev)
        lib = L.lib()
        dLdT = torch.empty_like(T)
        L.check("eik_obs_loss", lib.eik_obs_loss(T.numel(), L.dtype_code(T), L.ptr(T), L.ptr(T_obs), L.ptr(mask),
                                                 L.ptr(dLdT), L.ptr(self.scalars), L.ptr(self.scratch), st))
        dMp, dop, _ = E.adjoint(Mp, op, T, par, None, src, h, dLdT, src_t=src_t)
        if self.lam_tv > 0:
            ny, nx = T.shape
            for F, gF, w, off in ((Mp, dMp, I.G_WEIGHTS, 1), (op, dop, I.B_WEIGHTS, 2)):
                wt = (ctypes.c_double * len(w))(*w)
                L.check("eik_tv", lib.eik_tv(nx, ny, len(w), L.dtype_code(F), L.ptr(F), wt, self.lam_tv, L.ptr(gF),
                                             self.scalars.data_ptr() + 8 * off, L.ptr(self.scratch), st))
        dM, dom = E.project_backward(M, om, dMp, dop)
        self.enc.backward(dM, dom)
        return T, self.scalars.clone()

    def step(self, scene):
        """One Adam step on one scene (dict with X, y, src, h, T_obs, mask)."""
        T, s = self.gradients(scene["X"], scene["y"], scene["src"], scene["h"], scene["T_obs"], scene["mask"])
        self.enc.adam_step(self.lr)
        return s

    # -- several scenes of one size per step --------------------------------
    def _batch_plan(self, B, H, W, h, n_src):
        from .batched import Batch
        key = (B, H, W, float(h), int(n_src))
        if getattr(self, "_bkey", None) != key:
            self._batch = Batch([(W, H, h, n_src)] * B, dtype=torch.float32, device=self.enc.dev, max_rounds=4096)
            self._bkey = key
        return self._batch

    def predict_batch(self, X, y, srcs, h):
        """X (B, n_cov, H, W), y (B, n_global), srcs a list of B int32 source
        tensors of one length: the B scenes through the encoder, the
        projection and one batched solve (eik_forward_batched). Returns T
        (B, H, W) and the state the gradient needs."""
        self.enc.set_inputs(X, y)
        M, om = self.enc.forward()
        B, _, H, W = M.shape
        proj = [E.project(M[b], om[b]) for b in range(B)]
        Mp = torch.stack([q[0] for q in proj])
        op = torch.stack([q[1] for q in proj])
        src = torch.cat([t.to(torch.int32).reshape(-1) for t in srcs])
        bt = self._batch_plan(B, H, W, h, srcs[0].numel())
        T, par, _, _ = bt.forward(Mp.reshape(-1), op.reshape(-1), src, tol=self.tol)
        return T.view(B, H, W), (M, om, Mp, op, par, src, bt)

    def gradients_batch(self, X, y, srcs, h, T_obs, mask):
        """The hybrid gradient of the summed data term of B scenes (T_obs and
        mask (B, H, W)), accumulated into enc.grads; one batched adjoint."""
        T, (M, om, Mp, op, par, src, bt) = self.predict_batch(X, y, srcs, h)
        B, _, H, W = M.shape
        lib, st = L.lib(), L.stream_handle(self.enc.dev)
        T_obs, mask = T_obs.contiguous(), mask.contiguous()
        dLdT = torch.empty_like(T)
        L.check("eik_obs_loss", lib.eik_obs_loss(T.numel(), L.dtype_code(T), L.ptr(T), L.ptr(T_obs), L.ptr(mask),
                                                 L.ptr(dLdT), L.ptr(self.scalars), L.ptr(self.scratch), st))
        dMp, dop, _, _ = bt.backward(Mp.reshape(-1), op.reshape(-1), T.reshape(-1), par, None, src,
                                     dLdT.reshape(-1))
        dMp, dop = dMp.view(B, 3, H, W), dop.view(B, 2, H, W)
        if self.lam_tv > 0:
            for b in range(B):
                for F, gF, w, off in ((Mp[b], dMp[b], I.G_WEIGHTS, 1), (op[b], dop[b], I.B_WEIGHTS, 2)):
                    wt = (ctypes.c_double * len(w))(*w)
                    L.check("eik_tv", lib.eik_tv(W, H, len(w), L.dtype_code(F), L.ptr(F), wt, self.lam_tv, L.ptr(gF),
                                                 self.scalars.data_ptr() + 8 * off, L.ptr(self.scratch), st))
        back = [E.project_backward(M[b], om[b], dMp[b], dop[b]) for b in range(B)]
        self.enc.backward(torch.stack([q[0] for q in back]), torch.stack([q[1] for q in back]))
        return T, self.scalars.clone()

    def step_batch(self, scenes):
        """One Adam step on a list of scenes of one size (dicts as in step)."""
        X = torch.stack([sc["X"] for sc in scenes])
        y = torch.stack([sc["y"] for sc in scenes])
        T_obs = torch.stack([sc["T_obs"] for sc in scenes])
        mask = torch.stack([sc["mask"] for sc in scenes])
        T, s = self.gradients_batch(X, y, [sc["src"] for sc in scenes], scenes[0]["h"], T_obs, mask)
        self.enc.adam_step(self.lr)
        return s


def correlation(T, T_obs, mask):
    """Pearson correlation of predicted and observed arrival times over the
    observed nodes (the paper's evaluation metric)."""
    m = mask.bool() & torch.isfinite(T) & torch.isfinite(T_obs)
    a, b = T[m].double(), T_obs[m].double()
    a, b = a - a.mean(), b - b.mean()
    return float((a * b).sum() / torch.sqrt((a * a).sum() * (b * b).sum()))
