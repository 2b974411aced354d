"""Test infrastructure, not product code: plain float64 numpy references of
the inverse-problem pieces (Sec. 5, Eq. inverse_problem; App. learning
details, "Total Variation Regularization"; App. inverse problem experiments,
optimiser). Only tests/, smoke() and the benchmark's CPU baseline use it.

Readings where the paper is silent: gradients of the fields are forward
differences in grid units, zero across the last column and row; where a
node's gradient norm is 0 its term contributes the subgradient 0; the data
term is one half of the sum of squared residuals over the observed nodes.
"""
from __future__ import annotations

import numpy as np


def _diffs(F):
    """Forward differences of planes F [C, ny, nx] along x and y (zero at the
    last column / row)."""
    dx = np.zeros_like(F)
    dy = np.zeros_like(F)
    dx[:, :, :-1] = F[:, :, 1:] - F[:, :, :-1]
    dy[:, :-1, :] = F[:, 1:, :] - F[:, :-1, :]
    return dx, dy


def tv(F, weights):
    """R = sum_ij sqrt(sum_c w_c (dx_c^2 + dy_c^2)) and dR/dF (App. learning
    details: Frobenius norm of the metric's gradient with the off-diagonal
    weighted by 2, Euclidean norm of the drift's)."""
    F = np.asarray(F, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64).reshape(-1, 1, 1)
    dx, dy = _diffs(F)
    n = np.sqrt(np.sum(w * (dx * dx + dy * dy), axis=0))
    value = float(n.sum())
    inv = np.where(n > 0, 1.0 / np.where(n > 0, n, 1.0), 0.0)
    ax = w * dx * inv  # d n_ij / d (dx_c)_ij
    ay = w * dy * inv
    g = np.zeros_like(F)
    # (dx)_ij = F_(i+1,j) - F_(i,j): +ax at (i+1, j), -ax at (i, j)
    g[:, :, 1:] += ax[:, :, :-1]
    g[:, :, :-1] -= ax[:, :, :-1]
    g[:, 1:, :] += ay[:, :-1, :]
    g[:, :-1, :] -= ay[:, :-1, :]
    return value, g


def obs_loss(T, T_obs, mask):
    """L = 1/2 sum over observed finite nodes of (T - That)^2 and dL/dT."""
    T = np.asarray(T, dtype=np.float64)
    T_obs = np.asarray(T_obs, dtype=np.float64)
    use = (np.asarray(mask) != 0) & np.isfinite(T) & np.isfinite(T_obs)
    r = np.where(use, T - np.where(use, T_obs, 0.0), 0.0)
    return 0.5 * float(np.sum(r * r)), r


def clip_scale(grad_sq, max_norm):
    """Global-norm clipping factor min(1, max_norm / ||g||) (1 when off)."""
    if max_norm <= 0:
        return 1.0
    norm = float(np.sqrt(grad_sq))
    return 1.0 if norm <= max_norm else max_norm / norm


def param_step(method, p, g, m, v, lr, beta1=0.9, beta2=0.999, eps=1e-8, t=1, max_norm=0.0, grad_sq=0.0):
    """One step: method 0 projected gradient descent p - lr g, method 1 Adam
    with bias correction at step t. Returns new (p, m, v)."""
    g = np.asarray(g, dtype=np.float64) * clip_scale(grad_sq, max_norm)
    p = np.asarray(p, dtype=np.float64)
    if method == 0:
        return p - lr * g, m, v
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def tie_isotropic(M):
    """Projection onto isotropic metrics G = g I (the constraint of the
    isotropic recovery experiment, Sec. 5): the Frobenius-nearest g I to G is
    g = (m11 + m22) / 2, with m12 = 0."""
    M = np.asarray(M, dtype=np.float64)
    g = 0.5 * (M[0] + M[2])
    return np.stack([g, np.zeros_like(g), g])
