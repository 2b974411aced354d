"""Seeded synthetic inputs for the Randers eikonal solve.

This module builds input fields only. It holds none of the solver's arithmetic
and is the one piece shared by the oracle tests, the HIP tests, the smoke check
and the benchmark.

Recipe (numpy ``default_rng(seed)``; draw order per seed: f_l1, f_l2, f_theta,
f_wx, f_wy, then sources, then loss cells):

* a smooth field is a sum of 8 cosines with integer wave vectors in
  [-4, 4]^2 \\ {0}, N(0,1) amplitudes and U[0, 2pi) phases, evaluated at node
  positions (i h, j h) and min-max normalised to [0, 1];
* eigenvalues l = l_min (l_max / l_min)^f (log-uniform), angle theta = pi f;
* metric M = R(theta) diag(l1, l2) R(theta)^T stored as planes (m11, m12, m22);
* drift omega_raw = (2 f_wx - 1, 2 f_wy - 1) rescaled by one global factor so
  that max over nodes of |omega|_{M^-1} equals rho_max (feasible Randers data);
* the 2048^2 stress workload adds 4 sharp regions (Voronoi cells of 4 random
  sites), each adding its own angle offset U[0, pi) to theta.

The workloads stand in for the paper's synthetic timing problems (anisotropic
metrics, small or moderate drift, point ignitions); no dataset is used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    nx: int
    ny: int
    h: float
    M: np.ndarray          # (3, ny, nx) float64: m11, m12, m22
    omega: np.ndarray      # (2, ny, nx) float64: bx, by
    src_idx: np.ndarray    # (n_src,) int32 flat indices j*nx+i
    src_t: np.ndarray      # (n_src,) float64 source times
    loss_idx: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    name: str = ""
    seed: int = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def rounded(self, dtype) -> "Problem":
        """Inputs rounded to ``dtype`` and returned in float64 (what an FP32 run sees)."""
        return Problem(self.nx, self.ny, float(np.asarray(self.h, dtype)),
                       self.M.astype(dtype).astype(np.float64),
                       self.omega.astype(dtype).astype(np.float64),
                       self.src_idx.copy(), self.src_t.astype(dtype).astype(np.float64),
                       self.loss_idx.copy(), self.name, self.seed)


def fourier_field(rng: np.random.Generator, nx: int, ny: int, h: float,
                  n_modes: int = 8, kmax: int = 4) -> np.ndarray:
    ks = []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, size=2)
        if k[0] != 0 or k[1] != 0:
            ks.append(k)
    amp = rng.standard_normal(n_modes)
    phase = rng.uniform(0.0, 2 * np.pi, n_modes)
    x = np.arange(nx) * h
    y = np.arange(ny) * h
    X, Y = np.meshgrid(x, y)  # (ny, nx)
    f = np.zeros((ny, nx))
    for (kx, ky), a, p in zip(ks, amp, phase):
        f += a * np.cos(2 * np.pi * (kx * X + ky * Y) + p)
    lo, hi = f.min(), f.max()
    return (f - lo) / (hi - lo) if hi > lo else np.zeros_like(f)


def metric_from_eig(l1, l2, theta):
    c, s = np.cos(theta), np.sin(theta)
    return np.stack([l1 * c * c + l2 * s * s, (l1 - l2) * s * c, l1 * s * s + l2 * c * c])


def drift_inverse_norm(M: np.ndarray, w: np.ndarray) -> np.ndarray:
    """|w|_{M^-1} per node (used only to scale synthetic drift to a target)."""
    m11, m12, m22 = M
    det = m11 * m22 - m12 * m12
    return np.sqrt((w[0] ** 2 * m22 - 2 * w[0] * w[1] * m12 + w[1] ** 2 * m11) / det)


def random_fields(rng, nx, ny, h, l_min, l_max, rho_max, regions: int = 0):
    f1 = fourier_field(rng, nx, ny, h)
    f2 = fourier_field(rng, nx, ny, h)
    ft = fourier_field(rng, nx, ny, h)
    fwx = fourier_field(rng, nx, ny, h)
    fwy = fourier_field(rng, nx, ny, h)
    l1 = l_min * (l_max / l_min) ** f1
    l2 = l_min * (l_max / l_min) ** f2
    theta = np.pi * ft
    if regions:
        sites = rng.uniform(0.0, 1.0, size=(regions, 2)) * np.array([(nx - 1) * h, (ny - 1) * h])
        offs = rng.uniform(0.0, np.pi, size=regions)
        X, Y = np.meshgrid(np.arange(nx) * h, np.arange(ny) * h)
        d2 = np.stack([(X - sx) ** 2 + (Y - sy) ** 2 for sx, sy in sites])
        theta = theta + offs[np.argmin(d2, axis=0)]
    M = metric_from_eig(l1, l2, theta)
    w = np.stack([2 * fwx - 1, 2 * fwy - 1])
    if rho_max > 0:
        w = w * (rho_max / drift_inverse_norm(M, w).max())
    else:
        w = np.zeros_like(w)
    return M, w


def random_sources(rng, nx, ny, n_src):
    idx = rng.choice(nx * ny, size=n_src, replace=False)
    return np.sort(idx).astype(np.int32)


def random_loss_cells(rng, n, count, exclude):
    cand = np.setdiff1d(np.arange(n), exclude)
    return np.sort(rng.choice(cand, size=min(count, cand.size), replace=False)).astype(np.int32)


def make_problem(config: str, seed: int = 0, nx: int | None = None, ny: int | None = None) -> Problem:
    """The five workloads, by name:

    c1  64x64, FP64 run, l in [0.5, 2], rho_max 0.5, one source at (32, 32),
        64 loss cells;
    c2  512x512, FP32 run, l in [0.5, 2], rho_max 0.7, 4 random sources,
        256 loss cells;
    c3  2048x2048, FP32 run, l in [10^-0.5, 10^0.5] (ratio 10), rho_max 0.9,
        4 sharp regions, 16 random sources, dense loss;
    c4  one grid of the batched set: sides U{64..512} each, h = 1/(max side - 1),
        c1 ranges, 1-4 random sources; seed g gives grid g;
    c5  256x256, c1 ranges, 1-4 random sources.

    ``nx``/``ny`` override the size (the field recipe is unchanged) for the
    small parity cases that span several tiles and a ragged tail.
    """
    rng = np.random.default_rng(seed)
    if config == "c1":
        nx_, ny_, lmin, lmax, rho, reg = 64, 64, 0.5, 2.0, 0.5, 0
    elif config == "c2":
        nx_, ny_, lmin, lmax, rho, reg = 512, 512, 0.5, 2.0, 0.7, 0
    elif config == "c3":
        nx_, ny_, lmin, lmax, rho, reg = 2048, 2048, 10 ** -0.5, 10 ** 0.5, 0.9, 4
    elif config == "c4":
        nx_, ny_ = int(rng.integers(64, 513)), int(rng.integers(64, 513))
        lmin, lmax, rho, reg = 0.5, 2.0, 0.5, 0
    elif config == "c5":
        nx_, ny_, lmin, lmax, rho, reg = 256, 256, 0.5, 2.0, 0.5, 0
    else:
        raise ValueError(config)
    nx_ = nx or nx_
    ny_ = ny or ny_
    h = 1.0 / (max(nx_, ny_) - 1)
    M, w = random_fields(rng, nx_, ny_, h, lmin, lmax, rho, reg)
    if config == "c1":
        src = np.array([(ny_ // 2) * nx_ + nx_ // 2], np.int32)
        n_loss = 64
    elif config == "c2":
        src = random_sources(rng, nx_, ny_, 4)
        n_loss = 256
    elif config == "c3":
        src = random_sources(rng, nx_, ny_, 16)
        n_loss = 0
    else:
        src = random_sources(rng, nx_, ny_, int(rng.integers(1, 5)))
        n_loss = 0
    loss = random_loss_cells(rng, nx_ * ny_, n_loss, src) if n_loss else np.zeros(0, np.int32)
    return Problem(nx_, ny_, h, M, w, src, np.zeros(src.size), loss, config, seed)


def constant_problem(nx, ny, h, g11, g12, g22, bx, by, sources, src_t=None) -> Problem:
    """Constant metric and drift with explicit (i, j) point sources."""
    M = np.stack([np.full((ny, nx), g11), np.full((ny, nx), g12), np.full((ny, nx), g22)]).astype(np.float64)
    w = np.stack([np.full((ny, nx), bx), np.full((ny, nx), by)]).astype(np.float64)
    src = np.array([j * nx + i for i, j in sources], np.int32)
    t = np.zeros(src.size) if src_t is None else np.asarray(src_t, np.float64)
    return Problem(nx, ny, h, M, w, src, t, np.zeros(0, np.int32), "const", 0)


def batched_set(n_grids: int = 256, base_seed: int = 1000):
    """The batched workload: grid g uses seed base_seed + g."""
    return [make_problem("c4", base_seed + g) for g in range(n_grids)]
