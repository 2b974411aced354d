"""The gradient checks of the paper's validation section (Sec. 4, gradient
validation; App. gradient verification), run on the library's FP64 path:

* pointwise: central finite differences (eps = 1e-5) of a linear functional
  L = sum_i c_i T_i with respect to single parameters at random interior
  nodes, against the implicit gradient; a node counts only where the active
  stencils do not change under +-eps (differentiable there);
* random directions: directional derivatives along random unit directions in
  the metric's parameter space, by finite differences and by the gradient;
* stability: change of the gradient when 1 % Gaussian noise is added to the
  metric, over the whole field and entry by entry at interior nodes; the
  noise independent per node or spatially correlated.

Configurations follow the paper: isotropic (G = I, b = 0), anisotropic
(eigenvalues 2 and 0.5 at 30 degrees), drift (G = I, b = (0.15, 0.08)); one
source at the centre of an n x n grid.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import eikonal as E

CONFIGS = ("isotropic", "anisotropic", "drift")


def config_fields(name, n, device, dtype=torch.float64):
    if name == "anisotropic":
        l1, l2, th = 2.0, 0.5, math.radians(30.0)
        c, s = math.cos(th), math.sin(th)
        m11, m12, m22 = l1 * c * c + l2 * s * s, (l1 - l2) * c * s, l1 * s * s + l2 * c * c
    else:
        m11, m12, m22 = 1.0, 0.0, 1.0
    bx, by = (0.15, 0.08) if name == "drift" else (0.0, 0.0)
    M = torch.tensor([m11, m12, m22], dtype=dtype, device=device).view(3, 1, 1).expand(3, n, n).contiguous()
    om = torch.tensor([bx, by], dtype=dtype, device=device).view(2, 1, 1).expand(2, n, n).contiguous()
    return M, om


# Components perturbed per configuration (the paper's pointwise table):
# metric and drift, metric only, drift only.
PLANES = {"isotropic": ("M", "om"), "anisotropic": ("M",), "drift": ("om",)}


class Check:
    """Gradient checks of one configuration. ``tau`` (in units of h) switches
    to the soft-min mode: T and its gradient come from the smooth soft-min
    solve and its adjoint, and no finite difference is skipped (the soft
    update has no stencil switches)."""

    def __init__(self, name, n=64, seed=0, device="cuda", tau=None):
        self.dev = torch.device(device)
        self.n = n
        self.h = 1.0 / (n - 1)
        self.tau = None if tau is None else tau * self.h
        self.M, self.om = config_fields(name, n, self.dev)
        self.src = torch.tensor([(n // 2) * n + n // 2], dtype=torch.int32, device=self.dev)
        rng = np.random.default_rng(seed)
        self.c = torch.tensor(rng.uniform(0.0, 1.0, (n, n)), device=self.dev)
        self.rng = rng

    def solve(self, M, om):
        if self.tau is not None:
            T, _, conv = E.soft_solve(M, om, self.src, self.h, self.tau, tol=1e-14)
            if not conv:
                raise RuntimeError("soft-min solve did not settle")
            return T, None
        T, par, _, _ = E.solve(M, om, self.src, self.h, tol=0.0, levels=False)
        return T, par

    def fd(self, Mp, omp, Mm, omm, eps):
        """Central difference of L along a perturbation, with the two fields
        subtracted node by node before the weighted sum (summing first would
        cancel catastrophically); also whether the active stencils of both
        solves equal those of the unperturbed one."""
        Tp, pp = self.solve(Mp, omp)
        Tm, pm = self.solve(Mm, omm)
        d = torch.where(torch.isfinite(Tp) & torch.isfinite(Tm), Tp - Tm, torch.zeros_like(Tp))
        return float((self.c * d).sum()) / (2 * eps), pp, pm

    def grad(self, M, om):
        T, par = self.solve(M, om)
        if self.tau is not None:
            dM, dom, _ = E.soft_adjoint(M, om, T, self.src, self.h, self.tau, self.c, tol=1e-14)
        else:
            dM, dom, _ = E.adjoint(M, om, T, par, None, self.src, self.h, self.c)
        return dM, dom

    def pointwise(self, points=20, eps=1e-5, planes=("M", "om")):
        """Max relative error over sampled (plane, component, node) entries
        whose active stencils stay fixed under +-eps (every entry in the
        soft-min mode); returns (max_err, tested, skipped)."""
        dM, dom = self.grad(self.M, self.om)
        _, par0 = self.solve(self.M, self.om)
        errs, skipped = [], 0
        n = self.n
        while len(errs) < points:
            which = planes[self.rng.integers(len(planes))]
            base, g = (self.M, dM) if which == "M" else (self.om, dom)
            comp = int(self.rng.integers(base.shape[0]))
            j, i = (int(x) for x in self.rng.integers(2, n - 2, 2))
            an = float(g[comp, j, i])
            if abs(an) < 1e-8 * float(g.abs().max()):
                continue
            P, Q = base.clone(), base.clone()
            P[comp, j, i] += eps
            Q[comp, j, i] -= eps
            if which == "M":
                fd, pp, pm = self.fd(P, self.om, Q, self.om, eps)
            else:
                fd, pp, pm = self.fd(self.M, P, self.M, Q, eps)
            if par0 is not None and not (torch.equal(pp, par0) and torch.equal(pm, par0)):
                skipped += 1
                continue
            errs.append(abs(fd - an) / abs(an))
        return max(errs), len(errs), skipped

    def random_directions(self, count=100, eps=1e-5):
        """Fractions of random unit directions in the metric's parameter
        space whose finite-difference directional derivative is within 10 %
        and 1 % of the gradient's."""
        dM, _ = self.grad(self.M, self.om)
        errs = []
        for _ in range(count):
            d = torch.tensor(self.rng.normal(size=self.M.shape), device=self.dev)
            d /= d.norm()
            fd, _, _ = self.fd(self.M + eps * d, self.om, self.M - eps * d, self.om, eps)
            an = float((dM * d).sum())
            errs.append(abs(fd - an) / max(abs(an), 1e-300))
        errs = np.array(errs)
        return float((errs < 0.1).mean()), float((errs < 0.01).mean()), float(np.median(errs))

    def smoothed(self, K=16, sigma=0.01):
        """Gradient function averaged over K jittered copies of the metric
        (relative Gaussian jitter of size sigma, draws fixed once so the
        smoothed gradient is a deterministic function of the parameters)."""
        from .smoothing import Jitter
        n = self.n
        J = Jitter(K, n, n, self.h, 1, dtype=self.M.dtype, device=self.dev)
        xi_M = sigma * self.M.abs()[None] * torch.tensor(self.rng.normal(size=(K, 3, n, n)), device=self.dev)
        xi_om = torch.zeros((K, 2, n, n), dtype=self.M.dtype, device=self.dev)
        loss = lambda T: (float((self.c * T).sum()), self.c)

        def grad(M, om):
            gM, gom, _, _ = J.gradient(M, om, self.src, loss, xi_M, xi_om)
            return gM, gom
        return grad

    def noise_field(self, corr=None):
        """Standard Gaussian noise on the three metric planes: independent per
        node (corr None), or spatially correlated, white noise filtered by a
        Gaussian of standard deviation ``corr`` nodes and rescaled to unit
        variance per plane."""
        Z = self.rng.normal(size=self.M.shape)
        if corr:
            k = np.fft.fftfreq(self.n)
            g = np.exp(-0.5 * (2 * np.pi * corr) ** 2 * (k[:, None] ** 2 + k[None, :] ** 2))
            Z = np.real(np.fft.ifft2(np.fft.fft2(Z, axes=(1, 2)) * g, axes=(1, 2)))
            Z /= Z.std(axis=(1, 2), keepdims=True)
        return torch.tensor(Z, device=self.dev)

    def stability(self, trials=10, noise=0.01, rel_floor=1e-2, grad=None, corr=None):
        """Change of the metric gradient under relative Gaussian noise of the
        given size on the metric (kept SPD by the feasibility projection),
        independent per node or correlated over ``corr`` nodes (noise_field),
        averaged over trials: the relative L2 change of the whole gradient
        field, and the mean and median of the per-entry relative change at
        interior nodes whose unperturbed entry is at least rel_floor of the
        largest (the smaller entries sit in the shadow of the functional and
        make the ratio meaningless). ``grad`` replaces the plain gradient
        (e.g. by a smoothed one)."""
        grad = grad or self.grad
        dM0, _ = grad(self.M, self.om)
        n = self.n
        inner = torch.zeros_like(dM0, dtype=torch.bool)
        inner[:, 2:n - 2, 2:n - 2] = True
        sel = inner & (dM0.abs() >= rel_floor * float(dM0.abs().max()))
        field, mean_pt, med_pt = [], [], []
        for _ in range(trials):
            Z = self.noise_field(corr)
            Mn, omn = E.project(self.M * (1.0 + noise * Z), self.om)
            dM, _ = grad(Mn, omn)
            field.append(float((dM - dM0).norm() / dM0.norm()))
            r = ((dM - dM0).abs() / dM0.abs())[sel]
            mean_pt.append(float(r.mean()))
            med_pt.append(float(r.median()))
        return {"field_rel_l2": float(np.mean(field)), "interior_mean": float(np.mean(mean_pt)),
                "interior_median": float(np.mean(med_pt)), "entries": int(sel.sum()), "trials": trials}
