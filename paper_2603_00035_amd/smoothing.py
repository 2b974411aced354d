"""Gradient averaging under parameter jitter: the smooth alternative to the
piecewise-smooth solution operator that the paper names beside soft-min
stencil selection (Sec. 3, stencil boundaries and non-smoothness).

The solution operator T(theta) is smooth where the active stencils stay fixed
and only continuous where they switch, so the gradient of a loss jumps across
those boundaries. Averaging over K jittered copies of the parameters,

    g(theta) = 1/K sum_k d/dtheta L(T(P(theta + xi_k))),

estimates the gradient of the smoothed objective E_xi[L(T(P(theta + xi)))]
(P the feasibility projection, differentiated exactly), which varies
continuously with theta for a fixed set of draws xi_k.

The K copies are one batched launch (eik_forward_batched and
eik_backward_batched over K grids of the same size), followed by K
eik_project_backward calls; the draws are the caller's input.
"""
from __future__ import annotations

import torch

from . import eikonal as E
from .batched import Batch


class Jitter:
    """Plan for K jittered copies of one (nx, ny) grid with n_src sources."""

    def __init__(self, K, nx, ny, h, n_src, dtype=torch.float64, device="cuda", tol=0.0, max_rounds=4096):
        self.K, self.nx, self.ny, self.h = int(K), int(nx), int(ny), float(h)
        self.tol = float(tol)
        self.batch = Batch([(nx, ny, h, n_src)] * self.K, dtype=dtype, device=device, max_rounds=max_rounds)

    def gradient(self, M, om, src_idx, dLdT_of, xi_M, xi_om, src_t=None):
        """Mean over the copies of the gradient with respect to (M, om) of
        L(T(P(M + xi_M[k], om + xi_om[k]))), and the mean loss.

        dLdT_of(T) -> (L, dL/dT) is the loss, called once per copy on its
        (ny, nx) arrival times; xi_M (K, 3, ny, nx) and xi_om (K, 2, ny, nx)
        are the draws. Returns (gM, gom, mean L, list of the K fields T)."""
        K = self.K
        if xi_M.shape != (K, 3, self.ny, self.nx) or xi_om.shape != (K, 2, self.ny, self.nx):
            raise ValueError("jitter draws must be (K, 3, ny, nx) and (K, 2, ny, nx)")
        E._check_fields(M, om)
        raw = [(M + xi_M[k], om + xi_om[k]) for k in range(K)]
        proj = [E.project(Mk.contiguous(), ok.contiguous()) for Mk, ok in raw]
        Mp, op = self.batch.pack([p[0] for p in proj], [p[1] for p in proj])
        src = torch.cat([src_idx.to(torch.int32)] * K).contiguous()
        st = None if src_t is None else torch.cat([src_t.to(Mp.dtype)] * K).contiguous()
        T, par, _, _ = self.batch.forward(Mp, op, src, src_t=st, tol=self.tol)
        Ts = self.batch.unpack_nodes(T)
        losses, grads = zip(*(dLdT_of(Tk) for Tk in Ts))
        dLdT = torch.cat([g.reshape(-1).to(Mp.dtype) for g in grads]).contiguous()
        dM, dom, _, _ = self.batch.backward(Mp, op, T, par, None, src, dLdT)
        gMs, goms = self.batch.unpack_planes(dM, 3), self.batch.unpack_planes(dom, 2)
        gM = torch.zeros_like(M)
        gom = torch.zeros_like(om)
        for k, (Mk, ok) in enumerate(raw):
            a, b = E.project_backward(Mk.contiguous(), ok.contiguous(), gMs[k], goms[k])
            gM += a
            gom += b
        return gM / K, gom / K, sum(float(v) for v in losses) / K, Ts
