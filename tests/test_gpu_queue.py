"""GPU parity of the work-queue scheduler (one persistent launch whose waves
take flagged tiles from a device queue) against the oracle, on the same seeded
inputs and with the same tolerances as the round scheduler."""
import numpy as np
import pytest

import oracle
from synthetic.fields import make_problem
from tests.gpu_common import (FP32_GRAD_RTOL, check_levels_consistent, check_parent_choices, oracle_view, rel_err_cells, rel_l2,
                              say, to_dev)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def queue_tuning(th=64, cycles=2):
    from paper_2603_00035_amd import eikonal as E
    return E.tuning(tile_height=th, max_local_cycles=cycles, scheduler=2, fast_cold_start=0)  # the queue alone


def solve(p, dt, tol, tune, **kw):
    from paper_2603_00035_amd import eikonal as E
    M, om, src, st = to_dev(p, dt)
    T, par, lev, stats = E.solve(M, om, src, p.h, src_t=st, tol=tol, tune=tune, **kw)
    torch.cuda.synchronize()
    return T, par, lev, stats, (M, om, src, st)


@pytest.mark.parametrize("cfg,seed,nx,ny,th", [("c1", 0, None, None, 64), ("c2", 1, 70, 201, 32),
                                               ("c2", 2, 129, 65, 64), ("c1", 3, 130, 97, 32)])
def test_queue_fp64_matches_oracle(cfg, seed, nx, ny, th):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem(cfg, seed, nx=nx, ny=ny)
    say(f"[queue fp64] {cfg} seed={seed} {p.nx}x{p.ny} th={th}")
    T, par, lev, stats, (M, om, src, st) = solve(p, torch.float64, 0.0, queue_tuning(th))
    assert stats.converged and stats.sweep_launches == 1
    To, _, _ = oracle.forward(p)
    Tg = T.cpu().numpy()
    assert rel_err_cells(Tg, To, p.src_idx) <= 1e-12
    po, lo = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)
    assert np.array_equal(lev.cpu().numpy(), lo)
    g = np.random.default_rng(seed).uniform(-1, 1, To.shape)
    dMo, domo, dso = oracle.vjp(p, To, po, g)
    for tune in (None, queue_tuning(th)):  # round-scheduled and queue-scheduled adjoint
        dM, dom, ds = E.adjoint(M, om, T, par, lev, src, p.h, torch.tensor(g, device=T.device), src_t=st,
                                tune=tune)
        assert rel_l2([dM.cpu().numpy(), dom.cpu().numpy(), ds.cpu().numpy()], [dMo, domo, dso]) <= 1e-10


def test_queue_fp32_c2_matches_oracle():
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c2", 0)
    q = oracle_view(p, "f32")
    say("[queue fp32] 512x512 tol 1e-5")
    T, par, lev, stats, (M, om, src, st) = solve(p, torch.float32, 1e-5, queue_tuning(64))
    assert stats.converged
    To, _, _ = oracle.forward(q)
    Tg = T.cpu().numpy().astype(np.float64)
    err = rel_err_cells(Tg, To, p.src_idx)
    say(f"  max rel err {err:.2e}, visits/tiles {stats.rounds}, updates/cell {stats.cell_updates / p.n:.1f}")
    assert err <= 1e-5
    po, _ = oracle.parents_levels(q, To)
    assert check_parent_choices(q, To, po, par.cpu().numpy(), 1e-5) <= p.n // 100
    check_levels_consistent(par.cpu().numpy(), lev.cpu().numpy(), Tg)
    g = np.random.default_rng(0).uniform(0, 1, To.shape)
    dM, dom, ds = E.adjoint(M, om, T, par, lev, src, p.h, torch.tensor(g, dtype=torch.float32, device=T.device),
                            tune=queue_tuning(64))
    dMo, domo, dso = oracle.vjp(q, To, po, g)
    r = rel_l2([dM.cpu().numpy().astype(np.float64), dom.cpu().numpy().astype(np.float64),
                ds.cpu().numpy().astype(np.float64)], [dMo, domo, dso])
    say(f"  gradient rel L2 {r:.2e}")
    assert r <= FP32_GRAD_RTOL


def test_queue_warm_start_and_visit_budget():
    p = make_problem("c2", 5, nx=150, ny=140)
    say("[queue warm/budget] 150x140 fp64")
    To, _, _ = oracle.forward(p)
    T0 = torch.tensor(To * np.random.default_rng(0).uniform(0.7, 1.3, To.shape))
    T, _, _, stats, _ = solve(p, torch.float64, 0.0, queue_tuning(32), T_init=T0)
    assert stats.converged
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    # a visit budget of one round's worth of tiles: stops early, reports it, no error
    T, _, _, stats, _ = solve(p, torch.float64, 0.0, queue_tuning(64, 1), max_rounds=1)
    assert not stats.converged and stats.status == 1


def test_queue_batched_matches_oracle_per_grid():
    from paper_2603_00035_amd.batched import Batch
    from tests.test_gpu_batched import packed_inputs, uneven_set
    probs = uneven_set(12, 2100)
    say(f"[queue batched] {len(probs)} grids fp64")
    B = Batch([(p.nx, p.ny, p.h, p.src_idx.size) for p in probs], dtype=torch.float64, tune=queue_tuning(32),
              max_rounds=4096)
    M, om, src = packed_inputs(B, probs, torch.float64)
    T, par, lev, st = B.forward(M, om, src, tol=0.0)
    assert st.converged
    for g, p in enumerate(probs):
        To, _, _ = oracle.forward(p)
        assert rel_err_cells(B.unpack_nodes(T)[g].cpu().numpy(), To, p.src_idx) <= 1e-12, g
