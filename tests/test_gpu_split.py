"""GPU parity of the split update (2 or 4 lanes share one node's local update,
a tile then runs on that many waves) against the oracle, on the same seeded
inputs and with the same tolerances as the one-lane update."""
import numpy as np
import pytest

import oracle
from synthetic.fields import constant_problem, make_problem
from tests.gpu_common import check_parent_choices, oracle_view, rel_err_cells, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def split_tuning(lanes, th=64):
    from paper_2603_00035_amd import eikonal as E
    return E.tuning(tile_height=th, node_lanes=lanes)


@pytest.mark.parametrize("lanes", [2, 4])
@pytest.mark.parametrize("cfg,seed,nx,ny,th", [("c1", 0, None, None, 64), ("c2", 1, 70, 201, 32),
                                               ("c2", 2, 129, 65, 64), ("c1", 3, 130, 97, 32)])
def test_split_fp64_matches_oracle(cfg, seed, nx, ny, th, lanes):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem(cfg, seed, nx=nx, ny=ny)
    say(f"[split fp64] {cfg} seed={seed} {p.nx}x{p.ny} th={th} lanes={lanes}")
    M, om, src, st = to_dev(p, torch.float64)
    T, par, lev, stats = E.solve(M, om, src, p.h, src_t=st, tol=0.0, tune=split_tuning(lanes, th), levels=False)
    assert stats.converged and lev is None
    To, _, _ = oracle.forward(p)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    po, _ = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)
    g = np.random.default_rng(seed).uniform(-1, 1, To.shape)
    dM, dom, ds = E.adjoint(M, om, T, par, None, src, p.h, torch.tensor(g, device=T.device), src_t=st)
    dMo, domo, dso = oracle.vjp(p, To, po, g)
    assert rel_l2([dM.cpu().numpy(), dom.cpu().numpy(), ds.cpu().numpy()], [dMo, domo, dso]) <= 1e-10


@pytest.mark.parametrize("lanes", [2, 4])
def test_split_fp32_c2_matches_oracle_and_one_lane(lanes):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c2", 0)
    q = oracle_view(p, "f32")
    say(f"[split fp32] 512x512 tol 1e-5 lanes={lanes}")
    M, om, src, _ = to_dev(p, torch.float32)
    T, par, _, stats = E.solve(M, om, src, p.h, tol=1e-5, tune=split_tuning(lanes), levels=False)
    assert stats.converged
    To, _, _ = oracle.forward(q)
    err = rel_err_cells(T.double().cpu().numpy(), To, p.src_idx)
    say(f"  max rel err {err:.2e}, rounds {stats.rounds}, updates/cell {stats.cell_updates / p.n:.1f}")
    assert err <= 1e-5
    po, _ = oracle.parents_levels(q, To)
    assert check_parent_choices(q, To, po, par.cpu().numpy(), 1e-5) <= p.n // 100
    # at exact stationarity the split and one-lane updates agree to rounding
    T0, _, _, _ = E.solve(M, om, src, p.h, tol=0.0, tune=split_tuning(1), levels=False)
    Ts, _, _, _ = E.solve(M, om, src, p.h, tol=0.0, tune=split_tuning(lanes), levels=False)
    d = (T0.double() - Ts.double()).abs().max().item() / T0[torch.isfinite(T0)].abs().max().item()
    say(f"  one-lane vs split at tol 0: {d:.2e}")
    assert d <= 1e-6


def test_split_edges():
    from paper_2603_00035_amd import eikonal as E
    for nx, ny, srcs in [(1, 1, [(0, 0)]), (1, 70, [(0, 3)]), (70, 1, [(69, 0)]), (2, 2, [(0, 0), (1, 1)])]:
        p = constant_problem(nx, ny, 0.1, 1.3, 0.2, 0.7, 0.1, -0.05, srcs)
        say(f"[split edge] {nx}x{ny}")
        M, om, src, st = to_dev(p, torch.float64)
        for lanes in (2, 4):
            T, par, _, _ = E.solve(M, om, src, p.h, src_t=st, tol=0.0, tune=split_tuning(lanes), levels=False)
            To, _, _ = oracle.forward(p)
            assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
