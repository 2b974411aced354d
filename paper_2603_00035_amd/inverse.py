"""Recovery of metric and drift fields from observed arrival times (Sec. 5,
Eq. inverse_problem): minimise

    1/2 sum_{i observed} (T_i(theta) - That_i)^2 + lam_G R(G) + lam_b R(b)

with total-variation regularisers (App. learning details: Frobenius norm of
the metric's gradient with the off-diagonal weighted by 2, or of the gradient
of its matrix logarithm (Log-Euclidean variant), Euclidean norm of the
drift's) by projected gradient steps or Adam with global-norm clipping and
a learning-rate schedule (App. inverse problem experiments), then projection
onto the feasible set (SPD metric, |b|_{G^-1} < 1).

Every step of an iteration is a library call (include/eik.h,
include/eik_inverse.h): eik_forward, eik_obs_loss, eik_backward, eik_tv,
eik_sum_sq, eik_param_step, eik_tie_isotropic (isotropic recovery),
eik_project. This module only sequences them and holds the optimiser state;
with several fires (MultiRecovery) it also replicates the parameter planes
for the batched launch and sums the per-fire gradients.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _lib as L
from . import eikonal as E

G_WEIGHTS = (1.0, 2.0, 1.0)  # m11, m12, m22: Frobenius norm of the symmetric tensor's gradient
B_WEIGHTS = (1.0, 1.0)


@dataclass
class InverseConfig:
    lam_G: float = 1e-3
    lam_b: float = 1e-3
    method: str = "adam"          # "adam" or "gd" (projected gradient descent)
    lr_G: float = 1e-2            # step sizes of the paper's projected gradient descent
    lr_b: float = 5e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    max_norm: float = 0.0         # global-norm clipping of the full gradient (0: off)
    schedule: str = "cosine"      # "cosine" (to lr_min_frac of the step size) or "constant"
    lr_min_frac: float = 0.1
    free_metric: bool = True
    free_drift: bool = True
    isotropic: bool = False       # constrain the metric to G = g I (projection after each step)
    tv_metric: str = "frobenius"  # metric TV: "frobenius" (|grad G|_F) or "log_euclid" (|grad log G|_F)
    tol: float = 0.0              # forward solve tolerance of every iteration
    eig_min: float = 1e-3         # projection (eik_project)
    eig_max: float = 1e3
    eucl_clip: float = 1e3
    rho_max: float = 0.95


def lr_at(cfg: InverseConfig, lr: float, k: int, iters: int) -> float:
    """Step size of iteration k of iters under the schedule."""
    if cfg.schedule == "constant" or iters <= 1:
        return lr
    lo = cfg.lr_min_frac * lr
    return lo + 0.5 * (lr - lo) * (1.0 + math.cos(math.pi * k / (iters - 1)))


def obs_loss(T, T_obs, mask, scratch, value):
    """eik_obs_loss: returns dL/dT of L = 1/2 sum over observed nodes of
    (T - T_obs)^2 and writes L into the device double `value`."""
    dLdT = torch.empty_like(T)
    L.check("eik_obs_loss", L.lib().eik_obs_loss(T.numel(), L.dtype_code(T), L.ptr(T), L.ptr(T_obs), L.ptr(mask),
                                                 L.ptr(dLdT), value.data_ptr(), L.ptr(scratch),
                                                 L.stream_handle(T.device)))
    return dLdT


class Recovery:
    """State of one recovery run: parameters M (3, ny, nx) and omega (2, ny,
    nx) on the GPU, observations T_obs (ny, nx) with a uint8 mask, sources."""

    def __init__(self, M0, om0, src_idx, h, T_obs, mask, cfg: InverseConfig | None = None, src_t=None):
        E._check_fields(M0, om0)
        self.cfg = cfg or InverseConfig()
        self.M = M0.detach().clone().contiguous()
        self.om = om0.detach().clone().contiguous()
        self.src = src_idx
        self.src_t = src_t
        self.h = float(h)
        self.T_obs = T_obs.to(device=self.M.device, dtype=self.M.dtype).contiguous()
        self.mask = mask.to(device=self.M.device, dtype=torch.uint8).contiguous()
        self.ny, self.nx = self.M.shape[1:]
        self.dc = L.dtype_code(self.M)
        dev = self.M.device
        self.scratch = torch.empty(L.lib().eik_inv_scratch_bytes(), dtype=torch.uint8, device=dev)
        self.scalars = torch.zeros(4, dtype=torch.float64, device=dev)  # data loss, R(G), R(b), |g|^2
        self.mM = torch.zeros_like(self.M)
        self.vM = torch.zeros_like(self.M)
        self.mo = torch.zeros_like(self.om)
        self.vo = torch.zeros_like(self.om)
        self.t = 0
        self._stream = L.stream_handle(dev)
        if self.cfg.tv_metric not in ("frobenius", "log_euclid"):
            raise ValueError(f"tv_metric {self.cfg.tv_metric!r}: 'frobenius' or 'log_euclid'")
        self.tv_work = None
        if self.cfg.tv_metric == "log_euclid":
            nb = L.lib().eik_tv_log_euclid_work_bytes(self.nx, self.ny, self.dc)
            self.tv_work = torch.empty(nb, dtype=torch.uint8, device=dev)

    def _sp(self, k):
        return self.scalars.data_ptr() + 8 * k

    def _data_gradient(self):
        """Gradients (dL/dM, dL/domega) of the data term at the current
        parameters; the data loss goes to scalars[0]."""
        c = self.cfg
        lib, st = L.lib(), self._stream
        n = self.nx * self.ny
        T, par, _, _ = E.solve(self.M, self.om, self.src, self.h, src_t=self.src_t, tol=c.tol, levels=False)
        dLdT = torch.empty_like(T)
        L.check("eik_obs_loss", lib.eik_obs_loss(n, self.dc, L.ptr(T), L.ptr(self.T_obs), L.ptr(self.mask),
                                                 L.ptr(dLdT), self._sp(0), L.ptr(self.scratch), st))
        gM, gom, _ = E.adjoint(self.M, self.om, T, par, None, self.src, self.h, dLdT, src_t=self.src_t)
        return gM, gom

    def step(self, k: int = 0, iters: int = 1):
        """One iteration; returns the device tensor (data loss, lam_G R(G),
        lam_b R(b), squared gradient norm) of the parameters it started from."""
        c = self.cfg
        lib, st = L.lib(), self._stream
        n = self.nx * self.ny
        gM, gom = self._data_gradient()
        self.scalars[1:].zero_()
        if c.free_metric and c.lam_G > 0 and c.tv_metric == "log_euclid":
            L.check("eik_tv_log_euclid",
                    lib.eik_tv_log_euclid(self.nx, self.ny, self.dc, L.ptr(self.M), c.lam_G, L.ptr(gM), self._sp(1),
                                          L.ptr(self.tv_work), L.ptr(self.scratch), st))
        elif c.free_metric and c.lam_G > 0:
            w = (ctypes.c_double * 3)(*G_WEIGHTS)
            L.check("eik_tv", lib.eik_tv(self.nx, self.ny, 3, self.dc, L.ptr(self.M), w, c.lam_G, L.ptr(gM),
                                         self._sp(1), L.ptr(self.scratch), st))
        if c.free_drift and c.lam_b > 0:
            w = (ctypes.c_double * 2)(*B_WEIGHTS)
            L.check("eik_tv", lib.eik_tv(self.nx, self.ny, 2, self.dc, L.ptr(self.om), w, c.lam_b, L.ptr(gom),
                                         self._sp(2), L.ptr(self.scratch), st))
        groups = [(c.free_metric, self.M, gM, self.mM, self.vM, c.lr_G),
                  (c.free_drift, self.om, gom, self.mo, self.vo, c.lr_b)]
        for free, p, g, _, _, _ in groups:
            if free:
                L.check("eik_sum_sq", lib.eik_sum_sq(p.numel(), self.dc, L.ptr(g), self._sp(3), L.ptr(self.scratch),
                                                     st))
        self.t += 1
        method = 1 if c.method == "adam" else 0
        for free, p, g, m, v, lr in groups:
            if not free:
                continue
            L.check("eik_param_step",
                    lib.eik_param_step(p.numel(), self.dc, method, L.ptr(p), L.ptr(g), L.ptr(m), L.ptr(v),
                                       lr_at(c, lr, k, iters), c.beta1, c.beta2, c.eps, self.t, c.max_norm,
                                       self._sp(3), st))
        if c.isotropic:
            L.check("eik_tie_isotropic", lib.eik_tie_isotropic(n, self.dc, L.ptr(self.M), st))
        self.M, self.om = E.project(self.M, self.om, c.eig_min, c.eig_max, c.eucl_clip, c.rho_max)
        out = self.scalars.clone()
        return out

    def run(self, iters: int):
        """iters iterations; returns a (iters, 4) float64 CPU tensor of the
        per-iteration (data loss, lam_G R(G), lam_b R(b), |g|^2)."""
        hist = [self.step(k, iters) for k in range(iters)]
        return torch.stack(hist).cpu()


class MultiRecovery(Recovery):
    """Joint recovery from K fires on one grid (Sec. 5, multi-source recovery):
    fire f has its own ignition src[f] and observations T_obs[f] with mask
    mask[f], and the data term is the sum over the fires. The K forward
    solves and adjoints run as one batched launch (eik_forward_batched,
    eik_backward_batched over K copies of the parameter planes), then the
    per-fire gradients are summed; the rest of the iteration is Recovery's."""

    def __init__(self, M0, om0, srcs, h, T_obs, mask, cfg: InverseConfig | None = None):
        from .batched import Batch
        super().__init__(M0, om0, srcs[0], h, T_obs[0], mask[0], cfg)
        self.K = len(srcs)
        if T_obs.shape[0] != self.K or mask.shape[0] != self.K:
            raise ValueError("one observation field and one mask per fire")
        self.T_obs = T_obs.to(device=self.M.device, dtype=self.M.dtype).contiguous()
        self.mask = mask.to(device=self.M.device, dtype=torch.uint8).contiguous()
        self.src_all = torch.cat([s.to(device=self.M.device, dtype=torch.int32).reshape(-1) for s in srcs])
        self.batch = Batch([(self.nx, self.ny, self.h, int(s.numel())) for s in srcs], dtype=self.M.dtype,
                           device=self.M.device, max_rounds=4096)

    def _data_gradient(self):
        K, n = self.K, self.nx * self.ny
        lib, st = L.lib(), self._stream
        Mp = self.M.reshape(1, -1).expand(K, -1).contiguous().reshape(-1)
        op = self.om.reshape(1, -1).expand(K, -1).contiguous().reshape(-1)
        T, par, _, _ = self.batch.forward(Mp, op, self.src_all, tol=self.cfg.tol)
        dLdT = torch.empty_like(T)
        L.check("eik_obs_loss", lib.eik_obs_loss(K * n, self.dc, L.ptr(T), L.ptr(self.T_obs), L.ptr(self.mask),
                                                 L.ptr(dLdT), self._sp(0), L.ptr(self.scratch), st))
        dM, dom, _, _ = self.batch.backward(Mp, op, T, par, None, self.src_all, dLdT)
        gM = dM.view(K, 3, self.ny, self.nx).sum(0)
        gom = dom.view(K, 2, self.ny, self.nx).sum(0)
        return gM.contiguous(), gom.contiguous()
