"""Pins of the oracle's adjoint (Alg. backward) against exact identities and
finite differences. CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from synthetic.fields import Problem, constant_problem, make_problem, random_fields, random_sources

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def small_random(seed, n=20, rho=0.5, lo=0.5, hi=2.0, n_src=2):
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    M, w = random_fields(rng, n, n, h, lo, hi, rho)
    src = random_sources(rng, n, n, n_src)
    return Problem(n, n, h, M, w, src, rng.uniform(0, 0.05, src.size))


def solve(p):
    T, _, st = oracle.forward(p)
    assert st == 0
    par, lev = oracle.parents_levels(p, T)
    return T, par, lev


def test_w1_gradient():
    """The worked example embedded in a 2x2 grid: donors are sources with
    times 0 (node (0,0)) and 0.5 (node (0,1)); node (1,1) takes the W1 update."""
    w1 = json.load(open(os.path.join(GOLD, "w1_two_point.json")))
    p = constant_problem(2, 2, 1.0, 1, 0, 1, 0, 0, [(0, 0), (0, 1)], src_t=[0.0, 0.5])
    T, par, _ = solve(p)
    assert T[1, 1] == pytest.approx(w1["T0"], abs=1e-15)
    assert par[1, 1] == 1  # stencil k=1: neighbours (-1,0) and (-1,-1)
    g = np.zeros((2, 2))
    g[1, 1] = 1.0
    dM, dom, ds = oracle.vjp(p, T, par, g)
    assert dM[:, 1, 1] == pytest.approx(w1["dT_dm"], abs=1e-14)
    assert dom[:, 1, 1] == pytest.approx(w1["dT_db"], abs=1e-14)
    # weights on the donors: node (0,1) is neighbour 1 (T=0.5), node (0,0) is neighbour 2
    assert ds == pytest.approx([w1["weights"][1], w1["weights"][0]], abs=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_dot_product_jvp_vjp(seed):
    p = small_random(seed)
    T, par, _ = solve(p)
    rng = np.random.default_rng(100 + seed)
    g = rng.standard_normal(T.shape)
    dMi = rng.standard_normal(p.M.shape)
    domi = rng.standard_normal(p.omega.shape)
    dsi = rng.standard_normal(p.src_idx.size)
    dT = oracle.jvp(p, T, par, dMi, domi, dsi)
    dM, dom, ds = oracle.vjp(p, T, par, g)
    lhs = np.sum(g * dT)
    rhs = np.sum(dM * dMi) + np.sum(dom * domi) + np.sum(ds * dsi)
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_mass_conservation(seed):
    """Donor weights are non-negative and sum to one, so every unit of dL/dT
    reaches the sources: sum_s dL/dt_s = sum_i g_i."""
    p = small_random(seed, n_src=3)
    T, par, _ = solve(p)
    g = np.random.default_rng(seed).uniform(-1, 1, T.shape)
    _, _, ds = oracle.vjp(p, T, par, g)
    assert ds.sum() == pytest.approx(g.sum(), rel=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_euler_homogeneity_identity(seed):
    """T(a^2 G, a b, a t) = a T, differentiated at a = 1:
    sum [2 (m11 gm11 + m12 gm12 + m22 gm22) + b . gb] + sum_s t_s gt_s = sum_i g_i T_i."""
    p = small_random(seed)
    T, par, _ = solve(p)
    g = np.random.default_rng(seed).uniform(-1, 1, T.shape)
    dM, dom, ds = oracle.vjp(p, T, par, g)
    lhs = 2 * np.sum(p.M * dM) + np.sum(p.omega * dom) + np.sum(p.src_t * ds)
    assert lhs == pytest.approx(np.sum(g * T), rel=1e-12)


def test_lattice_ray_target_constant_medium():
    """On a lattice ray in a constant medium T_j = F(d) exactly, so the summed
    gradients are those of the closed form: sum dT/db = d, sum dT/dG = d d^T/(2|d|_G)."""
    n = 31
    h = 1.0 / (n - 1)
    G = (1.625, 0.6495190528383290, 0.875)
    b = (0.2, 0.1)
    p = constant_problem(n, n, h, *G, *b, [(15, 15)])
    T, par, _ = solve(p)
    for k, r in [(5, 10), (6, 9), (7, 12), (2, 11)]:
        i, j = 15 + r * oracle.NBX[k], 15 + r * oracle.NBY[k]
        g = np.zeros_like(T)
        g[j, i] = 1.0
        dM, dom, ds = oracle.vjp(p, T, par, g)
        d = np.array([(i - 15) * h, (j - 15) * h])
        nG = np.sqrt(G[0] * d[0] ** 2 + 2 * G[1] * d[0] * d[1] + G[2] * d[1] ** 2)
        assert dom[0].sum() == pytest.approx(d[0], abs=1e-12)
        assert dom[1].sum() == pytest.approx(d[1], abs=1e-12)
        assert dM[0].sum() == pytest.approx(d[0] ** 2 / (2 * nG), abs=1e-12)
        assert dM[1].sum() == pytest.approx(d[0] * d[1] / nG, abs=1e-12)
        assert dM[2].sum() == pytest.approx(d[1] ** 2 / (2 * nG), abs=1e-12)
        assert ds[0] == pytest.approx(1.0, abs=1e-12)


def test_psd_sign_of_metric_gradient():
    p = small_random(11)
    T, par, _ = solve(p)
    g = np.random.default_rng(0).uniform(0, 1, T.shape)
    dM, _, _ = oracle.vjp(p, T, par, g)
    a, c, d = dM[0], dM[1] / 2, dM[2]
    assert np.all(a >= -1e-15) and np.all(d >= -1e-15)
    assert np.all(a * d - c * c >= -1e-12 * (np.abs(a * d) + 1e-30))


def fd_check(p, T, par, cells, g, eps_rel=1e-5):
    """Central FD of L = <g, T> w.r.t. each stored scalar at each cell (eps as
    in Sec. 4.2's gradient table), kept only when the active-stencil map is
    unchanged at +-eps. The absolute slack is the FD rounding noise of L,
    about 1e-15 sum|g T| / eps."""
    dM, dom, ds = oracle.vjp(p, T, par, g)
    noise = 5e-15 * np.sum(np.abs(g * T))
    checked = 0
    for c in cells:
        j, i = divmod(int(c), p.nx)
        for arr, grad, k in [("M", dM, 0), ("M", dM, 1), ("M", dM, 2), ("omega", dom, 0), ("omega", dom, 1)]:
            base = getattr(p, arr)
            eps = eps_rel * max(1.0, abs(base[k, j, i]))
            vals = []
            same = True
            for s in (+1, -1):
                q = Problem(p.nx, p.ny, p.h, p.M.copy(), p.omega.copy(), p.src_idx, p.src_t)
                getattr(q, arr)[k, j, i] += s * eps
                Tq, _, _ = oracle.forward(q)
                pq, _ = oracle.parents_levels(q, Tq)
                same &= np.array_equal(pq, par)
                vals.append(np.sum(g * Tq))
            if not same:
                continue
            fd = (vals[0] - vals[1]) / (2 * eps)
            assert grad[k, j, i] == pytest.approx(fd, rel=1e-5, abs=noise / eps)
            checked += 1
    return checked


@pytest.mark.parametrize("seed", range(3))
def test_finite_differences_away_from_switches(seed):
    p = small_random(seed, n=16)
    T, par, _ = solve(p)
    rng = np.random.default_rng(seed)
    g = rng.uniform(0, 1, T.shape)
    cells = rng.choice(np.setdiff1d(np.arange(p.n), p.src_idx), 6, replace=False)
    assert fd_check(p, T, par, cells, g) >= 10


def test_c1_loss_gradient_fd():
    """The 64x64 workload's loss: L = mean over 64 cells of (T - T_target)^2."""
    p = make_problem("c1", 0)
    tgt = make_problem("c1", 1)
    T, par, _ = solve(p)
    Tt, _, _ = oracle.forward(Problem(p.nx, p.ny, p.h, tgt.M, tgt.omega, p.src_idx, p.src_t))
    g = np.zeros_like(T)
    g.flat[p.loss_idx] = 2 * (T.flat[p.loss_idx] - Tt.flat[p.loss_idx]) / p.loss_idx.size
    cells = p.loss_idx[:3]
    assert fd_check(p, T, par, cells, g) >= 5
