"""Seeded synthetic scenes for the covariate encoder: they stand in for the
Sim2Real-Fire scenes of the paper's wildfire experiments, which are not
available here.

This module builds inputs only (covariates, a hidden ground-truth metric,
an ignition point); it holds none of the solver's or the encoder's
arithmetic. Observed arrival times are made by the caller, by solving on the
hidden fields.

Recipe (numpy ``default_rng(seed)``; draw order: elevation, fuel, vegetation,
moisture fields, then wind direction, wind speed, temperature, humidity, then
the ignition node):

* spatial covariates X (4, n, n) in [0, 1]: elevation, fuel, vegetation,
  moisture, each a smooth 8-mode Fourier field (synthetic.fields);
* global covariates y (4,): cos and sin of the wind direction U[0, 2 pi),
  wind speed U[0.2, 1], humidity U[0, 1] (temperature is drawn and unused);
* hidden spread speed s = 0.6 + 0.9 fuel (1 - 0.5 moisture) + 0.3 vegetation
  - 0.2 humidity; slope direction from the elevation gradient, with spread
  along the slope faster by a = 1 + 1.5 |grad e| / max |grad e|; metric
  G = R diag(1 / (a s)^2, 1 / s^2) R^T with R along the slope;
* hidden drift b against the wind (spread downwind is faster), scaled so
  that max |b|_{G^-1} = 0.6 wind speed;
* one ignition node drawn uniformly from the central 80 % of the domain.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .fields import drift_inverse_norm, fourier_field, metric_from_eig


@dataclass
class Scene:
    n: int
    h: float
    X: np.ndarray        # (4, n, n) spatial covariates
    y: np.ndarray        # (4,) global covariates
    M: np.ndarray        # (3, n, n) hidden metric
    omega: np.ndarray    # (2, n, n) hidden drift
    src_idx: np.ndarray  # (1,) int32 ignition node
    seed: int = 0


def scene(seed: int, n: int = 64) -> Scene:
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    elev, fuel, veg, moist = (fourier_field(rng, n, n, h) for _ in range(4))
    wd = rng.uniform(0.0, 2 * np.pi)
    ws = rng.uniform(0.2, 1.0)
    _temp = rng.uniform(0.0, 1.0)
    hum = rng.uniform(0.0, 1.0)
    j, i = (int(v) for v in rng.integers(int(0.1 * n), int(0.9 * n), 2))
    s = 0.6 + 0.9 * fuel * (1.0 - 0.5 * moist) + 0.3 * veg - 0.2 * hum
    gy, gx = np.gradient(elev, h)
    gn = np.hypot(gx, gy)
    a = 1.0 + 1.5 * gn / max(gn.max(), 1e-12)
    M = metric_from_eig(1.0 / (a * s) ** 2, 1.0 / s ** 2, np.arctan2(gy, gx))
    w = -np.stack([np.full((n, n), np.cos(wd)), np.full((n, n), np.sin(wd))])
    w *= 0.6 * ws / drift_inverse_norm(M, w).max()
    X = np.stack([elev, fuel, veg, moist])
    y = np.array([np.cos(wd), np.sin(wd), ws, hum])
    return Scene(n, h, X, y, M, w, np.array([j * n + i], np.int32), seed)
