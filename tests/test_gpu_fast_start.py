"""GPU parity of the FAST cold start (restricted-candidate min sweeps before
the full ones): one wave per tile (mode 1) and four waves sweeping the four
directions of a tile at once (mode 2). Both end with full rounds, so the field
and the active stencils must equal the oracle's fixed point."""
import numpy as np
import pytest

import oracle
from synthetic.fields import Problem, make_problem
from tests.gpu_common import FP32_GRAD_RTOL, check_parent_choices, loss_grad_cells, oracle_view, rel_err_cells, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def tune(fast, th=64, sched=1, cycles=1):
    from paper_2603_00035_amd import eikonal as E
    return E.tuning(tile_height=th, fast_cold_start=fast, scheduler=sched, max_local_cycles=cycles)


@pytest.mark.parametrize("fast", [1, 2])
@pytest.mark.parametrize("cfg,seed,nx,ny,th,sched,cycles", [
    ("c1", 0, None, None, 64, 1, 1), ("c2", 1, 70, 201, 32, 1, 2), ("c2", 2, 257, 130, 64, 2, 1),
    ("c3", 3, 300, 260, 64, 1, 1), ("c3", 4, 129, 333, 32, 2, 2)])
def test_fast_start_fp64_is_the_fixed_point(fast, cfg, seed, nx, ny, th, sched, cycles):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem(cfg, seed, nx=nx, ny=ny)
    say(f"[fast {fast}] {cfg} seed={seed} {p.nx}x{p.ny} th={th} sched={sched} cycles={cycles}")
    M, om, src, st = to_dev(p, torch.float64)
    T, par, lev, s = E.solve(M, om, src, p.h, src_t=st, tol=0.0, tune=tune(fast, th, sched, cycles), levels=False)
    torch.cuda.synchronize()
    assert s.converged
    To, _, _ = oracle.forward(p)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    po, _ = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)


@pytest.mark.parametrize("fast", [1, 2])
def test_fast_start_with_levels_falls_back_to_one_wave(fast):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c2", 6, nx=140, ny=90)
    say(f"[fast {fast}] levels requested 140x90")
    M, om, src, st = to_dev(p, torch.float64)
    T, par, lev, s = E.solve(M, om, src, p.h, src_t=st, tol=0.0, tune=tune(fast), levels=True)
    To, _, _ = oracle.forward(p)
    po, lo = oracle.parents_levels(p, To)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    assert np.array_equal(lev.cpu().numpy(), lo)


@pytest.mark.parametrize("fast", [1, 2])
def test_fast_start_fp32_c2_and_loss_gradient(fast):
    """FP32 to 1e-5 and the gradient of the 256-cell loss (the FP32 parity
    recipe of the default path)."""
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c2", 0)
    q = oracle_view(p, "f32")
    say(f"[fast {fast}] c2 512x512 FP32 tol 1e-5, 256 loss cells")
    M, om, src, st = to_dev(p, torch.float32)
    T, par, _, s = E.solve(M, om, src, p.h, tol=1e-5, tune=tune(fast), levels=False)
    assert s.converged
    To, _, _ = oracle.forward(q)
    Tg = T.cpu().numpy().astype(np.float64)
    err = rel_err_cells(Tg, To, p.src_idx)
    say(f"  max rel err {err:.2e}, rounds {s.rounds}, updates/cell {s.cell_updates / p.n:.1f}")
    assert err <= 1e-5
    po, _ = oracle.parents_levels(q, To)
    assert check_parent_choices(q, To, po, par.cpu().numpy(), 1e-5) <= p.n // 100
    tgt = make_problem("c2", 1).rounded(np.float32)
    Tt, _, _ = oracle.forward(Problem(q.nx, q.ny, q.h, tgt.M, tgt.omega, q.src_idx, q.src_t))
    gg = loss_grad_cells(Tg, p.loss_idx, Tt)
    dM, dom, ds = E.adjoint(M, om, T, par, None, src, p.h, torch.tensor(gg, dtype=torch.float32, device=T.device))
    dMo, domo, _ = oracle.vjp(q, To, po, loss_grad_cells(To, p.loss_idx, Tt))
    r = rel_l2([dM.cpu().numpy().astype(np.float64), dom.cpu().numpy().astype(np.float64)], [dMo, domo])
    say(f"  gradient rel L2 {r:.2e}")
    assert r <= FP32_GRAD_RTOL
    # the mixed-precision path with this cold start meets 1e-4 on the same loss
    M6, om6 = M.double(), om.double()
    Tm, parm, _, _ = E.solve_mixed(M6, om6, src, p.h, tol=1e-5, tune32=tune(fast), levels=False)
    gm = torch.tensor(loss_grad_cells(Tm.cpu().numpy(), p.loss_idx, Tt), device=M.device)
    dMm, domm, _ = E.adjoint_mixed(M6, om6, Tm, parm, src, p.h, gm)
    rm = rel_l2([dMm.cpu().numpy(), domm.cpu().numpy()], [dMo, domo])
    say(f"  mixed precision: gradient rel L2 {rm:.2e}")
    assert rm <= 1e-4


def test_fast_cd_in_the_mixed_path():
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c3", 7, nx=320, ny=288)
    say("[fast 2] mixed path 320x288 stress recipe tol 0")
    M, om, src, _ = to_dev(p, torch.float64)
    T, par, _, (s32, s64) = E.solve_mixed(M, om, src, p.h, tol=0.0, tol32=1e-5, tune32=tune(2), levels=False)
    assert s64.converged
    To, _, _ = oracle.forward(p)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    po, _ = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)
