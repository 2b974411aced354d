"""Pins of the inverse-problem oracle (CPU): closed forms of the total
variation, finite differences of every gradient, and the optimiser's known
trajectories."""
import numpy as np
import pytest

from oracle import inverse_ref as I


def test_tv_of_a_step_edge_is_jump_times_length():
    ny, nx, k = 7, 9, 4
    F = np.ones((1, ny, nx))
    F[:, :, k:] = 3.0
    val, _ = I.tv(F, [1.0])
    assert val == pytest.approx(2.0 * ny)  # one jump of 2 per row, between columns k-1 and k


def test_tv_of_a_ramp_closed_form():
    ny, nx, a, b = 6, 8, 0.3, -0.7
    j, i = np.mgrid[0:ny, 0:nx]
    F = (a * i + b * j)[None].astype(np.float64)
    val, _ = I.tv(F, [1.0])
    want = (nx - 1) * (ny - 1) * np.hypot(a, b) + (ny - 1) * abs(b) + (nx - 1) * abs(a)
    assert val == pytest.approx(want, rel=1e-12)


def test_plane_weight_scales_its_norm():
    rng = np.random.default_rng(0)
    P = rng.normal(size=(1, 5, 6))
    Z = np.zeros_like(P)
    G = np.concatenate([Z, P, Z])  # only the off-diagonal varies
    vG, _ = I.tv(G, [1.0, 2.0, 1.0])
    vP, _ = I.tv(P, [1.0])
    assert vG == pytest.approx(np.sqrt(2.0) * vP, rel=1e-12)


@pytest.mark.parametrize("planes,weights", [(1, [1.0]), (2, [1.0, 1.0]), (3, [1.0, 2.0, 1.0])])
def test_tv_gradient_matches_central_differences(planes, weights):
    rng = np.random.default_rng(planes)
    F = rng.normal(size=(planes, 5, 7))
    _, g = I.tv(F, weights)
    eps = 1e-6
    for c, jj, ii in [(0, 0, 0), (planes - 1, 4, 6), (0, 2, 3), (planes - 1, 1, 5), (planes // 2, 4, 0)]:
        Fp, Fm = F.copy(), F.copy()
        Fp[c, jj, ii] += eps
        Fm[c, jj, ii] -= eps
        fd = (I.tv(Fp, weights)[0] - I.tv(Fm, weights)[0]) / (2 * eps)
        assert g[c, jj, ii] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_tv_subgradient_is_zero_on_flat_regions():
    F = np.full((2, 4, 5), 1.5)
    val, g = I.tv(F, [1.0, 1.0])
    assert val == 0.0 and not np.any(g)


def test_obs_loss_value_gradient_and_mask():
    rng = np.random.default_rng(3)
    T = rng.uniform(0, 2, (4, 6))
    To = rng.uniform(0, 2, (4, 6))
    mask = (rng.uniform(size=(4, 6)) < 0.5).astype(np.uint8)
    T[0, 0], mask[0, 0] = np.inf, 1  # an unreached observed node contributes nothing
    val, g = I.obs_loss(T, To, mask)
    use = (mask != 0) & np.isfinite(T)
    assert val == pytest.approx(0.5 * np.sum((T[use] - To[use]) ** 2))
    assert np.all(g[~use] == 0)
    k = tuple(np.argwhere(use)[0])
    Tp, Tm = T.copy(), T.copy()
    Tp[k] += 1e-6
    Tm[k] -= 1e-6
    fd = (I.obs_loss(Tp, To, mask)[0] - I.obs_loss(Tm, To, mask)[0]) / 2e-6
    assert g[k] == pytest.approx(fd, rel=1e-6)


def test_gradient_descent_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.5, 1.0, -4.0])
    q, _, _ = I.param_step(0, p, g, None, None, lr=0.1)
    assert np.allclose(q, [0.95, -2.1, 0.9])


def test_adam_moves_lr_per_step_under_a_constant_gradient():
    # with bias correction, m_hat = g and v_hat = g^2 at every step of a
    # constant gradient, so each step moves by lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.5, 1e-3, -4.0])
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 6):
        p, m, v = I.param_step(1, p, g, m, v, lr=0.01, t=t, eps=0.0)
    assert np.allclose(p, np.array([1.0, -2.0, 0.5]) - 5 * 0.01 * np.sign(g), rtol=0, atol=1e-12)


def test_clipping_caps_the_global_norm():
    g = np.array([3.0, 4.0])  # norm 5
    q, _, _ = I.param_step(0, np.zeros(2), g, None, None, lr=1.0, max_norm=1.0, grad_sq=25.0)
    assert np.linalg.norm(q) == pytest.approx(1.0)
    q, _, _ = I.param_step(0, np.zeros(2), g, None, None, lr=1.0, max_norm=10.0, grad_sq=25.0)
    assert np.allclose(-q, g)


def test_isotropic_tie_is_the_frobenius_nearest_isotropic_metric():
    rng = np.random.default_rng(11)
    M = rng.normal(size=(3, 4, 5))
    P = I.tie_isotropic(M)
    assert np.array_equal(I.tie_isotropic(P), P)  # a projection
    gs = np.linspace(-4, 4, 80001)
    for j, i in [(0, 0), (3, 4), (2, 1)]:
        m11, m12, m22 = M[:, j, i]
        # brute force over g of || G - g I ||_F^2 (the off-diagonal counts twice)
        d = (m11 - gs) ** 2 + 2 * m12 ** 2 + (m22 - gs) ** 2
        assert P[0, j, i] == pytest.approx(gs[np.argmin(d)], abs=1e-4)
        assert P[1, j, i] == 0.0 and P[0, j, i] == P[2, j, i]


# --- Log-Euclidean TV (App. learning details, Total Variation Regularization) --

def _spd_field(rng, ny, nx, iso_frac=0.0):
    A = rng.normal(size=(ny, nx, 2, 2))
    G = A @ np.swapaxes(A, -1, -2) + 0.2 * np.eye(2)
    iso = rng.uniform(size=(ny, nx)) < iso_frac
    g = rng.uniform(0.5, 2.0, size=(ny, nx))
    G[iso] = g[iso][:, None, None] * np.eye(2)
    return np.stack([G[..., 0, 0], G[..., 0, 1], G[..., 1, 1]]), G


def test_log_spd2_matches_scipy_logm():
    import scipy.linalg
    import torch
    rng = np.random.default_rng(1)
    M, G = _spd_field(rng, 6, 7, iso_frac=0.2)
    P = I.log_spd2(torch.tensor(M)).numpy()
    for j in range(6):
        for i in range(7):
            L = scipy.linalg.logm(G[j, i]).real
            assert np.allclose([P[0, j, i], P[1, j, i], P[2, j, i]], [L[0, 0], L[0, 1], L[1, 1]], atol=1e-13)


def test_log_euclid_tv_of_isotropic_fields_is_tv_of_log_g():
    """G = g I: log G = log(g) I, so |grad log G|_F = sqrt(2) |grad log g|."""
    rng = np.random.default_rng(2)
    g = rng.uniform(0.5, 3.0, size=(5, 8))
    M = np.stack([g, 0 * g, g])
    val, _ = I.tv_log_euclid(M)
    vlog, _ = I.tv(np.log(g)[None], [1.0])
    assert val == pytest.approx(np.sqrt(2.0) * vlog, rel=1e-12)


def test_log_euclid_tv_invariances():
    """Invariant under one rotation applied at every node (G -> Q G Q^T) and
    under one scale (log(a G) = log G + log(a) I, constant over the grid),
    neither of which holds for the Frobenius variant."""
    rng = np.random.default_rng(3)
    M, G = _spd_field(rng, 5, 6)
    v0, _ = I.tv_log_euclid(M)
    c, s = np.cos(0.7), np.sin(0.7)
    Q = np.array([[c, -s], [s, c]])
    GR = Q @ G @ Q.T
    v1, _ = I.tv_log_euclid(np.stack([GR[..., 0, 0], GR[..., 0, 1], GR[..., 1, 1]]))
    v2, _ = I.tv_log_euclid(3.7 * M)
    assert v1 == pytest.approx(v0, rel=1e-12)
    assert v2 == pytest.approx(v0, rel=1e-12)
    vf0, _ = I.tv(M, [1.0, 2.0, 1.0])
    vf2, _ = I.tv(3.7 * M, [1.0, 2.0, 1.0])
    assert vf2 == pytest.approx(3.7 * vf0, rel=1e-12)


def test_log_euclid_tv_gradient_matches_central_differences():
    """Every stored scalar (m12 enters both off-diagonal entries), including
    isotropic nodes where the eigenvalues coincide."""
    rng = np.random.default_rng(4)
    M, _ = _spd_field(rng, 4, 5, iso_frac=0.3)
    _, g = I.tv_log_euclid(M)
    eps = 1e-6
    for c in range(3):
        for j in range(4):
            for i in range(5):
                Mp, Mm = M.copy(), M.copy()
                Mp[c, j, i] += eps
                Mm[c, j, i] -= eps
                fd = (I.tv_log_euclid(Mp)[0] - I.tv_log_euclid(Mm)[0]) / (2 * eps)
                assert g[c, j, i] == pytest.approx(fd, rel=1e-5, abs=1e-7), (c, j, i)
