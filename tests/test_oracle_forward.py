"""Pins of the oracle's forward solve against facts the paper and the
mathematics fix (closed forms, brute force, invariants). CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from synthetic.fields import constant_problem, make_problem, metric_from_eig, Problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --- local updates --------------------------------------------------------

def test_w1_two_point_value_and_weights():
    w1 = gold("w1_two_point.json")
    a = w1["inputs"]
    ok, t, lam = oracle.two_point(a["G"], a["b"], a["h"], a["kp"], a["kq"], a["Tp"], a["Tq"])
    assert ok
    assert t == pytest.approx(w1["T0"], abs=1e-15)
    assert lam / lam.sum() == pytest.approx(w1["weights"], abs=1e-14)
    # both one-point candidates are larger, so the two-point update wins
    assert oracle.one_point(a["G"], a["b"], a["h"], a["kp"], a["Tp"]) == pytest.approx(w1["one_point_candidates"][0])
    assert oracle.one_point(a["G"], a["b"], a["h"], a["kq"], a["Tq"]) == pytest.approx(w1["one_point_candidates"][1])


@pytest.mark.parametrize("seed", range(6))
def test_two_point_matches_hopf_lax_scan(seed):
    """A valid two-point candidate is the interior minimum over the donor
    segment (envelope form of Eq. two_point); an invalid one has its minimum
    at an end point or violates causality."""
    rng = np.random.default_rng(seed)
    for _ in range(40):
        l1, l2 = rng.uniform(0.3, 3.0, 2)
        G = metric_from_eig(l1, l2, rng.uniform(0, np.pi))
        G = [float(x) for x in G]
        det = G[0] * G[2] - G[1] ** 2
        bdir = rng.standard_normal(2)
        rho = np.sqrt((bdir[0] ** 2 * G[2] - 2 * bdir[0] * bdir[1] * G[1] + bdir[1] ** 2 * G[0]) / det)
        b = bdir / rho * rng.uniform(0, 0.8)
        h = float(rng.uniform(0.01, 1.0))
        k = int(rng.integers(0, 8))
        Tp, Tq = rng.uniform(0, 1, 2)
        ok, t, lam = oracle.two_point(G, b, h, k, (k + 1) % 8, Tp, Tq)
        v, tt = oracle.hopf_lax_two_point(G, b, h, k, (k + 1) % 8, Tp, Tq)
        if ok:
            assert t == pytest.approx(v, abs=1e-9 * max(1, abs(v)))
            assert tt == pytest.approx(lam[1] / lam.sum(), abs=1e-4)
        elif lam.min() < 0 and 1e-3 < tt < 1 - 1e-3:
            pytest.fail("interior minimum rejected by the barycentric test")


# --- constant media: closed form, lattice rays, sandwich ------------------

def test_drift_asymmetry_39_21():
    d = gold("drift_asymmetry.json")
    n, (si, sj) = d["grid"], d["source"]
    p = constant_problem(n, n, 1.0, 1, 0, 1, d["b"][0], d["b"][1], [(si, sj)])
    T, _, st = oracle.forward(p)
    assert st == 0
    assert T[sj, si + 30] == pytest.approx(d["T_plus30"], abs=1e-12)
    assert T[sj, si - 30] == pytest.approx(d["T_minus30"], abs=1e-12)


CONST_CASES = [
    (1.0, 0.0, 1.0, 0.0, 0.0),          # isotropic
    (4.0, 0.0, 0.25, 0.0, 0.0),         # diagonal anisotropy (App. forward solver validation)
    (2.125, 1.875, 2.125, 0.0, 0.0),    # rotated 45 deg, eigenvalues 4 and 0.25
    (1.0, 0.0, 1.0, 0.3, 0.0),          # constant drift
    (1.625, 0.6495190528383290, 0.875, 0.2, 0.1),  # combined: eig 2, 0.5 at 30 deg, b=(0.2,0.1)
]


@pytest.mark.parametrize("case", CONST_CASES)
def test_constant_medium_lattice_rays_and_sandwich(case):
    n = 41
    h = 1.0 / (n - 1)
    p = constant_problem(n, n, h, *case, [(20, 20)])
    T, _, st = oracle.forward(p)
    assert st == 0
    F = oracle.closed_form(p, [(20, 20)])
    # the 8 lattice rays from the source are exact (one-point chains)
    for k in range(8):
        for r in range(1, 21):
            i, j = 20 + r * oracle.NBX[k], 20 + r * oracle.NBY[k]
            assert T[j, i] == pytest.approx(F[j, i], rel=1e-12, abs=1e-14)
    # sandwich: F(x - s) <= T <= Dijkstra on the 8-neighbour graph
    D = oracle.dijkstra(p)
    assert np.all(T >= F - 1e-12)
    assert np.all(T <= D + 1e-12)


def test_rotated_generator_g12():
    """App. forward solver validation: eigenvalues 4, 0.25 at 45 degrees give g12 = 1.875."""
    g = metric_from_eig(4.0, 0.25, np.pi / 4)
    assert g[1] == pytest.approx(1.875, abs=1e-15)
    assert g[0] == pytest.approx(2.125) and g[2] == pytest.approx(2.125)


def test_isotropic_refinement_soft_table():
    """Table convergence: error against |x - x0| decreases with refinement and
    has the paper's order of magnitude (the source position is unstated)."""
    ref = gold("convergence_table.json")
    errs = []
    for N in ref["N"][:4]:
        h = 1.0 / N
        c = N // 2
        p = constant_problem(N + 1, N + 1, h, 1, 0, 1, 0, 0, [(c, c)])
        T, _, _ = oracle.forward(p)
        F = oracle.closed_form(p, [(c, c)])
        errs.append(np.linalg.norm(T - F) / np.linalg.norm(F))
    assert all(a > b for a, b in zip(errs, errs[1:]))
    for e, r in zip(errs, ref["rel_L2"]):
        assert r / 4 < e < r * 4
    rate = -np.polyfit(np.log(ref["N"][:4]), np.log(errs), 1)[0]
    assert 0.4 < rate < 1.1


def test_three_sources_min_distance():
    """App. forward solver validation 'Multiple Ignition Points': sources at
    (N/4,N/4), (N/4,3N/4), (3N/4,N/2); the solution is bounded below by the
    minimum distance and close to it."""
    N = 100
    srcs = [(N // 4, N // 4), (N // 4, 3 * N // 4), (3 * N // 4, N // 2)]
    p = constant_problem(N + 1, N + 1, 1.0 / N, 1, 0, 1, 0, 0, srcs)
    T, _, _ = oracle.forward(p)
    F = oracle.closed_form(p, srcs)
    assert np.all(T >= F - 1e-12)
    rel = np.linalg.norm(T - F) / np.linalg.norm(F)
    assert rel < 0.01


# --- brute force and fixed-point properties on random media ---------------

def small_random(seed, n=16, rho=0.5, lo=0.5, hi=2.0, n_src=2):
    from synthetic.fields import random_fields, random_sources
    rng = np.random.default_rng(seed)
    h = 1.0 / (n - 1)
    M, w = random_fields(rng, n, n, h, lo, hi, rho)
    src = random_sources(rng, n, n, n_src)
    return Problem(n, n, h, M, w, src, np.zeros(src.size))


@pytest.mark.parametrize("seed", range(4))
def test_one_point_only_equals_dijkstra(seed):
    p = small_random(seed)
    T1, _, st = oracle.forward(p, one_point_only=True)
    assert st == 0
    D = oracle.dijkstra(p)
    assert np.allclose(T1, D, rtol=1e-12, atol=1e-14)
    T, _, _ = oracle.forward(p)
    assert np.all(T <= D + 1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_gauss_seidel_and_jacobi_reach_same_fixed_point(seed):
    p = small_random(seed, n=24)
    Tg, _, sg = oracle.forward(p)
    Tj, _, sj = oracle.forward(p, mode="jacobi")
    assert sg == 0 and sj == 0
    assert np.allclose(Tg, Tj, rtol=1e-13, atol=1e-15)


def test_fixed_point_is_stationary_and_c1_converges():
    p = make_problem("c1", 0)
    T, sweeps, st = oracle.forward(p)
    assert st == 0 and sweeps < 40
    for c in np.random.default_rng(0).choice(p.n, 200, replace=False):
        if c in set(p.src_idx):
            continue
        v, code = oracle.local_update(p, T, c)
        assert v == T.flat[c] and code < 16
    # the all-node evaluation agrees with the one-node one and leaves a zero
    # residual at every reached non-source node
    va, ca = oracle.local_update_all(p, T)
    m = np.isfinite(T)
    m.flat[p.src_idx] = False
    assert np.array_equal(va[m], T[m])
    for c in np.random.default_rng(1).choice(p.n, 50, replace=False):
        assert (va.flat[c], int(ca.flat[c])) == oracle.local_update(p, T, c)


def test_grid_spacing_scaling_and_homogeneity():
    p = small_random(7, n=20)
    T, _, _ = oracle.forward(p)
    q = Problem(p.nx, p.ny, 2.5 * p.h, p.M, p.omega, p.src_idx, p.src_t)
    T2, _, _ = oracle.forward(q)
    assert np.allclose(T2, 2.5 * T, rtol=1e-12)
    a = 1.7
    r = Problem(p.nx, p.ny, p.h, a * a * p.M, a * p.omega, p.src_idx, a * np.array([0.0, 0.3]))
    T3, _, _ = oracle.forward(r)
    p2 = Problem(p.nx, p.ny, p.h, p.M, p.omega, p.src_idx, np.array([0.0, 0.3]))
    T4, _, _ = oracle.forward(p2)
    assert np.allclose(T3, a * T4, rtol=1e-12)


def test_warm_start_overwrite_reaches_cold_fixed_point():
    p = small_random(3, n=24)
    T, _, _ = oracle.forward(p)
    rng = np.random.default_rng(1)
    for init in (np.zeros_like(T), T * rng.uniform(0.5, 1.5, T.shape), np.full_like(T, 10.0)):
        Tw, _, st = oracle.forward(p, T_init=init)
        assert st == 0
        assert np.allclose(Tw, T, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("stress", [False, True])
def test_parents_and_levels_define_a_causal_dag(stress):
    """Alg. backward's ordering argument: every donor of an active update has a
    strictly smaller arrival time. The stress media (eigenvalue ratio 10, drift
    0.9) make causality rejection of two-point candidates active."""
    if stress:
        p = small_random(5, n=32, n_src=3, rho=0.9, lo=10 ** -0.5, hi=10 ** 0.5)
    else:
        p = small_random(5, n=24, n_src=3)
    T, _, _ = oracle.forward(p)
    par, lev = oracle.parents_levels(p, T)
    srcs = set(int(s) for s in p.src_idx)
    nx = p.nx
    for c in range(p.n):
        if c in srcs:
            assert par.flat[c] == oracle.SOURCE and lev.flat[c] == 0
            continue
        code = int(par.flat[c])
        assert code < 16
        i, j = c % nx, c // nx
        ks = [code, (code + 1) % 8] if code < 8 else [code - 8]
        dl = []
        for k in ks:
            d = (j + oracle.NBY[k]) * nx + i + oracle.NBX[k]
            assert T.flat[d] < T.flat[c]
            dl.append(lev.flat[d])
        assert lev.flat[c] == 1 + max(dl)
