"""Pins of the oracle's feasibility projection (App. learning details,
"Feasibility Projections"). CPU only."""
import numpy as np
import pytest

import oracle
from synthetic.fields import drift_inverse_norm, metric_from_eig

KW = dict(eig_min=1e-3, eig_max=1e3, eucl_clip=1e3, rho_max=0.95)


def rand_inputs(rng, n, feasible):
    if feasible:
        l1, l2 = rng.uniform(0.1, 5, n), rng.uniform(0.1, 5, n)
    else:
        l1, l2 = rng.uniform(-2, 5, n), rng.uniform(1e-5, 2e3, n)
    M = metric_from_eig(l1, l2, rng.uniform(0, np.pi, n))
    w = rng.standard_normal((2, n))
    if feasible:
        w *= (rng.uniform(0, 0.9, n) / drift_inverse_norm(M, w))
    else:
        w *= rng.uniform(0, 3, n)
    return M, w


def eigs(M):
    tr, dif = M[0] + M[2], M[0] - M[2]
    disc = np.sqrt(dif ** 2 + 4 * M[1] ** 2)
    return 0.5 * (tr + disc), 0.5 * (tr - disc)


def test_identity_when_feasible():
    M, w = rand_inputs(np.random.default_rng(0), 500, True)
    Mo, wo = oracle.project(M, w, **KW)
    assert np.array_equal(Mo, M) and np.array_equal(wo, w)


def test_bounds_and_idempotence():
    M, w = rand_inputs(np.random.default_rng(1), 2000, False)
    Mo, wo = oracle.project(M, w, **KW)
    lp, lm = eigs(Mo)
    assert np.all(lm >= KW["eig_min"] * (1 - 1e-9)) and np.all(lp <= KW["eig_max"] * (1 + 1e-9))
    assert np.all(drift_inverse_norm(Mo, wo) <= KW["rho_max"] * (1 + 1e-12))
    M2, w2 = oracle.project(Mo, wo, **KW)
    assert np.allclose(M2, Mo, rtol=1e-9, atol=1e-12) and np.allclose(w2, wo, rtol=1e-9, atol=1e-12)


def test_rotation_equivariance():
    rng = np.random.default_rng(2)
    M, w = rand_inputs(rng, 300, False)
    a = rng.uniform(0, 2 * np.pi)
    c, s = np.cos(a), np.sin(a)
    R = np.array([[c, -s], [s, c]])

    def rot(M, w):
        G = np.array([[M[0], M[1]], [M[1], M[2]]]).transpose(2, 0, 1)
        Gr = R @ G @ R.T
        return np.stack([Gr[:, 0, 0], Gr[:, 0, 1], Gr[:, 1, 1]]), R @ w

    Mo, wo = oracle.project(M, w, **KW)
    Mr, wr = oracle.project(*rot(M, w), **KW)
    Mo_r, wo_r = rot(Mo, wo)
    assert np.allclose(Mr, Mo_r, rtol=1e-9, atol=1e-9)
    assert np.allclose(wr, wo_r, rtol=1e-9, atol=1e-9)


def test_projected_drift_defines_positive_finsler_norm():
    """|b|_{G^-1} < 1 is exactly the condition for F(v) = |v|_G + b.v > 0 (v != 0)."""
    M, w = rand_inputs(np.random.default_rng(3), 200, False)
    Mo, wo = oracle.project(M, w, **KW)
    ang = np.linspace(0, 2 * np.pi, 361)
    V = np.stack([np.cos(ang), np.sin(ang)])
    for c in range(Mo.shape[1]):
        g11, g12, g22 = Mo[:, c]
        F = np.sqrt(g11 * V[0] ** 2 + 2 * g12 * V[0] * V[1] + g22 * V[1] ** 2) + wo[0, c] * V[0] + wo[1, c] * V[1]
        assert F.min() > 0


def test_vjp_matches_finite_differences():
    rng = np.random.default_rng(4)
    M, w = rand_inputs(rng, 64, False)
    gM, gw = rng.standard_normal(M.shape), rng.standard_normal(w.shape)
    dM, dw = oracle.project_vjp(M, w, gM, gw, **KW)
    eps = 1e-6
    for arr, grad in ((M, dM), (w, dw)):
        for k in range(arr.shape[0]):
            for c in range(0, arr.shape[1], 5):
                ap, am = arr.copy(), arr.copy()
                ap[k, c] += eps
                am[k, c] -= eps
                Lp = sum(np.sum(x * y) for x, y in zip(oracle.project(ap if arr is M else M, ap if arr is w else w, **KW), (gM, gw)))
                Lm = sum(np.sum(x * y) for x, y in zip(oracle.project(am if arr is M else M, am if arr is w else w, **KW), (gM, gw)))
                assert grad[k, c] == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-5, abs=1e-6)
