"""GPU parity of the full-update visits in which four waves sweep the four
directions of a tile at once (full_waves = 4): cold starts with and without
the restricted-candidate phase, warm starts from perturbed fields (values move
both ways), and the FP64 phase of the mixed-precision solve."""
import numpy as np
import pytest

import oracle
from synthetic.fields import make_problem
from tests.gpu_common import rel_err_cells, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def tune(fast, th=64, cycles=1):
    from paper_2603_00035_amd import eikonal as E
    return E.tuning(tile_height=th, fast_cold_start=fast, max_local_cycles=cycles, full_waves=4)


@pytest.mark.parametrize("fast", [0, 2])
@pytest.mark.parametrize("cfg,seed,nx,ny,th,cycles", [
    ("c1", 0, None, None, 64, 1), ("c2", 1, 70, 201, 32, 2), ("c2", 2, 257, 130, 64, 1),
    ("c3", 3, 300, 260, 64, 1), ("c3", 4, 129, 333, 32, 2)])
def test_four_wave_full_visits_fp64(fast, cfg, seed, nx, ny, th, cycles):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem(cfg, seed, nx=nx, ny=ny)
    say(f"[full waves] fast={fast} {cfg} seed={seed} {p.nx}x{p.ny} th={th} cycles={cycles}")
    M, om, src, st = to_dev(p, torch.float64)
    T, par, _, s = E.solve(M, om, src, p.h, src_t=st, tol=0.0, tune=tune(fast, th, cycles), levels=False)
    torch.cuda.synchronize()
    assert s.converged
    To, _, _ = oracle.forward(p)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    po, _ = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)


@pytest.mark.parametrize("lo,hi", [(0.7, 1.3), (0.95, 1.05)])
def test_four_wave_full_visits_warm_start(lo, hi):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c3", 8, nx=220, ny=190)
    say(f"[full waves] warm start from To x U({lo}, {hi})")
    M, om, src, st = to_dev(p, torch.float64)
    To, _, _ = oracle.forward(p)
    T0 = torch.tensor(To * np.random.default_rng(1).uniform(lo, hi, To.shape), device=M.device)
    T, par, _, s = E.solve(M, om, src, p.h, src_t=st, T_init=T0, tol=0.0, tune=tune(0), levels=False)
    assert s.converged
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12


def test_four_wave_full_visits_in_the_mixed_path():
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c3", 9, nx=300, ny=280)
    say("[full waves] mixed path 300x280 tol 0")
    M, om, src, _ = to_dev(p, torch.float64)
    T, par, _, (s32, s64) = E.solve_mixed(M, om, src, p.h, tol=0.0, tol32=1e-5, tune32=tune(2), tune=tune(0),
                                          levels=False)
    assert s64.converged
    To, _, _ = oracle.forward(p)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    po, _ = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)
