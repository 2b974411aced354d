"""Batched GPU version of the synthetic field recipe in fields.py (same
distributions, torch random streams), used to produce training sets for the
learned warm start quickly. Input construction only; no solver arithmetic."""
from __future__ import annotations

import math

import torch

_KV = [(kx, ky) for kx in range(-4, 5) for ky in range(-4, 5) if kx or ky]


def fourier_fields(gen, B, nx, ny, h, n_modes=8, device="cuda"):
    kv = torch.tensor(_KV, dtype=torch.float32, device=device)
    idx = torch.randint(0, len(_KV), (B, n_modes), generator=gen, device=device)
    k = kv[idx]  # (B, m, 2)
    amp = torch.randn(B, n_modes, generator=gen, device=device)
    ph = torch.rand(B, n_modes, generator=gen, device=device) * (2 * math.pi)
    x = torch.arange(nx, device=device, dtype=torch.float32) * h
    y = torch.arange(ny, device=device, dtype=torch.float32) * h
    f = torch.zeros(B, ny, nx, device=device)
    for m in range(n_modes):
        arg = 2 * math.pi * (k[:, m, 0, None, None] * x[None, None, :] + k[:, m, 1, None, None] * y[None, :, None])
        f += amp[:, m, None, None] * torch.cos(arg + ph[:, m, None, None])
    lo = f.amin(dim=(1, 2), keepdim=True)
    hi = f.amax(dim=(1, 2), keepdim=True)
    return (f - lo) / (hi - lo).clamp_min(1e-30)


def random_batch(seed, B, nx=256, ny=256, l_min=0.5, l_max=2.0, rho_max=0.5, max_src=4, device="cuda"):
    """B problems of the warm-start workload: returns M (B,3,ny,nx), omega
    (B,2,ny,nx), src (B,max_src) int32 with -1 for unused slots, h (float)."""
    gen = torch.Generator(device=device).manual_seed(seed)
    h = 1.0 / (max(nx, ny) - 1)
    f1, f2, ft, fwx, fwy = (fourier_fields(gen, B, nx, ny, h, device=device) for _ in range(5))
    l1 = l_min * (l_max / l_min) ** f1
    l2 = l_min * (l_max / l_min) ** f2
    th = math.pi * ft
    c, s = torch.cos(th), torch.sin(th)
    M = torch.stack([l1 * c * c + l2 * s * s, (l1 - l2) * s * c, l1 * s * s + l2 * c * c], dim=1)
    w = torch.stack([2 * fwx - 1, 2 * fwy - 1], dim=1)
    det = M[:, 0] * M[:, 2] - M[:, 1] ** 2
    rho = torch.sqrt((w[:, 0] ** 2 * M[:, 2] - 2 * w[:, 0] * w[:, 1] * M[:, 1] + w[:, 1] ** 2 * M[:, 0]) / det)
    w = w * (rho_max / rho.amax(dim=(1, 2)))[:, None, None, None]
    n_src = torch.randint(1, max_src + 1, (B,), generator=gen, device=device)
    perm = torch.argsort(torch.rand(B, nx * ny, generator=gen, device=device), dim=1)[:, :max_src]
    slot = torch.arange(max_src, device=device)[None, :]
    src = torch.where(slot < n_src[:, None], perm, torch.full_like(perm, -1)).to(torch.int32)
    return M.contiguous(), w.contiguous(), src.contiguous(), h
