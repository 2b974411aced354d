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


def log_spd2(M):
    """Matrix logarithm of 2x2 SPD metrics given as stored planes (m11, m12,
    m22) [3, ...], as torch float64 planes (p11, p12, p22) of log G.

    For a 2x2 matrix with eigenvalues t +- d (t half the trace, d half the
    eigenvalue gap) any function f satisfies f(G) = a I + b (G - t I) with
    a = (f(t + d) + f(t - d)) / 2 and b = (f(t + d) - f(t - d)) / (2 d); for
    f = log, a = log(det G) / 2 and b = atanh(d / t) / d, which tends to
    1 / t as d -> 0 (the series 1 / t (1 + x^2 / 3 + x^4 / 5), x = d / t,
    is used below d / t = 1e-3, written in d^2 so that its derivative stays
    finite where the eigenvalues coincide). Differentiable with autograd."""
    import torch
    m11, m12, m22 = M[0], M[1], M[2]
    t = 0.5 * (m11 + m22)
    q = (0.5 * (m11 - m22)) ** 2 + m12 * m12  # d^2, free of the square root's kink at 0
    a = 0.5 * torch.log(m11 * m22 - m12 * m12)
    x2 = q / (t * t)
    small = x2 < 1e-6
    xs = torch.sqrt(torch.where(small, torch.full_like(x2, 0.25), x2))  # finite gradients where unused
    b = torch.where(small, (1.0 + x2 / 3.0 + x2 * x2 / 5.0) / t, torch.atanh(xs) / (xs * t))
    return torch.stack([a + b * (m11 - t), b * m12, a + b * (m22 - t)])


def tv_log_euclid(M):
    """Log-Euclidean TV of a metric field (App. learning details, Total
    Variation Regularization): R = sum_ij |grad log G_ij|_F, the Frobenius
    norm of the forward differences of log G (off-diagonal weighted by 2 in
    the squared norm, as for the Frobenius variant), and dR/d(m11, m12, m22)
    with respect to the stored scalars (m12 enters both off-diagonal entries)."""
    import torch
    Mt = torch.tensor(np.asarray(M, dtype=np.float64), requires_grad=True)
    P = log_spd2(Mt)
    value, gP = tv(P.detach().numpy(), [1.0, 2.0, 1.0])
    P.backward(torch.from_numpy(gP))
    return value, Mt.grad.numpy()
