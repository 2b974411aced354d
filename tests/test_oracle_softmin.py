"""Pins of the oracle's soft-min mode (the smooth alternative to stencil
selection named in Sec. 3.3): each stencil contributes the Hopf-Lax minimum
over its segment, a node the soft minimum -tau log sum exp(-H_k / tau) over its
eight stencils. Pinned by a closed form on a line, the tau -> 0 limit of the
hard solver, exact homogeneity, local partial derivatives against central
differences, mass conservation of the adjoint, and central differences of the
whole solve at random interior entries with none skipped (the soft update is
continuously differentiable, so no stencil switch needs excluding)."""
import numpy as np

import oracle
from synthetic.fields import Problem, constant_problem, make_problem

NBX = (-1, -1, -1, 0, 1, 1, 1, 0)
NBY = (1, 0, -1, -1, -1, 0, 1, 1)


def test_line_closed_form():
    # on a line only the left and right neighbours exist, each the endpoint of
    # two stencils: downstream of the source T_i = T_{i-1} + h - tau ln 2 up
    # to terms of order exp(-2 h / tau) from the downstream neighbour
    h, n = 0.1, 40
    tau = h / 10
    p = constant_problem(n, 1, h, 1.0, 0.0, 1.0, 0.0, 0.0, [(0, 0)])
    T, _, st = oracle.soft_forward(p, tau)
    assert st == 0
    assert np.max(np.abs(T[0] - np.arange(n) * (h - tau * np.log(2)))) < n * h * np.exp(-2 * h / tau)


def test_limit_of_the_hard_solver():
    # isotropic medium, central source: the soft field lies below the hard one
    # (a soft minimum is below the minimum) by at most ln 2 tau per step, and
    # by exactly that along the axes, 16 steps to the edge midpoints
    p = constant_problem(33, 33, 1 / 32, 1.0, 0.0, 1.0, 0.0, 0.0, [(16, 16)])
    Th, _, _ = oracle.forward(p)
    for tau in (1e-4 / 32, 1e-5 / 32):
        Ts, _, st = oracle.soft_forward(p, tau)
        assert st == 0
        gap = Th - Ts
        assert gap.min() >= 0.0
        assert abs(gap.max() / (16 * tau * np.log(2)) - 1) < 1e-3


def test_homogeneity_is_exact():
    # (G, b, t_s, tau) -> (4 G, 2 b, 2 t_s, 2 tau) doubles every candidate and
    # the soft minimum; all scalings are powers of two, so the field doubles bit
    # for bit
    p = make_problem("c1", 0, nx=24, ny=24)
    tau = 0.1 * p.h
    T1, _, _ = oracle.soft_forward(p, tau)
    q = Problem(p.nx, p.ny, p.h, 4 * p.M, 2 * p.omega, p.src_idx, 2 * p.src_t)
    T2, _, _ = oracle.soft_forward(q, 2 * tau)
    assert np.array_equal(T2, 2 * T1)


def test_local_partials_match_central_differences():
    p = make_problem("c2", 3, nx=24, ny=24)
    tau = 0.2 * p.h
    T, _, _ = oracle.soft_forward(p, tau)
    rng = np.random.default_rng(0)
    eps = 1e-6
    worst = 0.0
    for _ in range(40):
        c = int(rng.integers(p.nx + 1, p.n - p.nx - 1))
        _, coef, dth = oracle.soft_local(p, T, tau, c)
        i, j = c % p.nx, c // p.nx
        for k in range(8):
            nb = (j + NBY[k]) * p.nx + i + NBX[k]
            Tp, Tm = T.copy(), T.copy()
            Tp.flat[nb] += eps
            Tm.flat[nb] -= eps
            fd = (oracle.soft_local(p, Tp, tau, c)[0] - oracle.soft_local(p, Tm, tau, c)[0]) / (2 * eps)
            worst = max(worst, abs(fd - coef[k]))
        assert abs(coef.sum() - 1.0) < 1e-12  # shifting every neighbour shifts the node
        for a in range(5):
            arr = (p.M if a < 3 else p.omega).copy()
            comp = a if a < 3 else a - 3
            vals = []
            for s in (eps, -eps):
                P = arr.copy()
                P[comp].flat[c] += s
                q = Problem(p.nx, p.ny, p.h, P if a < 3 else p.M, P if a >= 3 else p.omega, p.src_idx, p.src_t)
                vals.append(oracle.soft_local(q, T, tau, c)[0])
            worst = max(worst, abs((vals[0] - vals[1]) / (2 * eps) - dth[a]))
    assert worst < 1e-7


def test_adjoint_conserves_mass():
    # the neighbour derivatives of every non-source node sum to 1, so the
    # source derivatives carry the whole loss: sum_s dL/dt_s = sum_i g_i
    p = make_problem("c2", 4, nx=28, ny=20)
    tau = 0.2 * p.h
    T, _, _ = oracle.soft_forward(p, tau)
    g = np.random.default_rng(1).uniform(0, 1, T.shape)
    _, _, ds = oracle.soft_vjp(p, T, tau, g)
    assert abs(ds.sum() - g[np.isfinite(T)].sum()) < 1e-10 * g.sum()


def test_vjp_matches_central_differences_at_every_sampled_entry():
    for cfg, seed in (("c1", 0), ("c2", 1)):
        p = make_problem(cfg, seed, nx=32, ny=32)
        tau = 0.1 * p.h
        T, _, st = oracle.soft_forward(p, tau, tol=0.0, max_sweeps=4000)
        assert st == 0
        c = np.random.default_rng(seed + 1).uniform(0, 1, T.shape)
        dM, dom, _ = oracle.soft_vjp(p, T, tau, c)
        rng = np.random.default_rng(seed + 2)
        eps = 1e-6
        for _ in range(12):
            which = int(rng.integers(5))
            arr = p.M if which < 3 else p.omega
            comp = which if which < 3 else which - 3
            j, i = (int(x) for x in rng.integers(2, p.nx - 2, 2))
            vals = []
            for s in (eps, -eps):
                P = arr.copy()
                P[comp, j, i] += s
                q = Problem(p.nx, p.ny, p.h, P if which < 3 else p.M, P if which >= 3 else p.omega, p.src_idx,
                            p.src_t)
                Tq, _, _ = oracle.soft_forward(q, tau, tol=0.0, max_sweeps=4000)
                vals.append(float(np.sum(c * (Tq - T))))
            fd = (vals[0] - vals[1]) / (2 * eps)
            an = (dM if which < 3 else dom)[comp, j, i]
            assert abs(fd - an) <= 1e-5 * abs(an) + 1e-12, (cfg, which, j, i, fd, an)


def _tie_gradients(dt, tau=None):
    """dT_c/dt_A for the node c midway between two sources A and B of an
    isotropic medium, with t_A = dt and t_B = 0: the hard update (oracle's
    solve, stencils and VJP) or the soft one at tau."""
    n, h = 17, 1 / 16
    p0 = constant_problem(n, n, h, 1.0, 0.0, 1.0, 0.0, 0.0, [(2, 8), (14, 8)])
    p = Problem(p0.nx, p0.ny, p0.h, p0.M, p0.omega, p0.src_idx, np.array([dt, 0.0]))
    g = np.zeros((n, n))
    g[8, 8] = 1.0
    if tau is None:
        T, _, _ = oracle.forward(p)
        par, _ = oracle.parents_levels(p, T)
        return oracle.vjp(p, T, par, g)[2][0]
    T, _, st = oracle.soft_forward(p, tau)
    assert st == 0
    return oracle.soft_vjp(p, T, tau, g)[2][0]


def test_soft_gradient_is_continuous_where_the_hard_one_jumps():
    # at a tie between two sources the hard node takes one source's path: its
    # derivative in t_A jumps from 1 to 0; the soft one passes through 1/2
    # (the two paths are mirror images) and changes linearly in the gap
    tau = 0.1 / 16
    for d in (1e-5, 1e-7):
        assert _tie_gradients(-d) == 1.0 and _tie_gradients(d) == 0.0
    lo5, hi5 = _tie_gradients(-1e-5, tau), _tie_gradients(1e-5, tau)
    lo7, hi7 = _tie_gradients(-1e-7, tau), _tie_gradients(1e-7, tau)
    assert abs((lo5 + hi5) / 2 - 0.5) < 1e-12 and abs((lo7 + hi7) / 2 - 0.5) < 1e-12
    assert 0.0 < lo7 - hi7 < lo5 - hi5 < 1e-2
    assert abs((lo5 - hi5) / (lo7 - hi7) / 100 - 1) < 1e-3
