"""GPU parity of the adjoint visits in which four waves sweep the four
directions of a tile at once (adjoint_waves = 4) against the oracle's
vector-Jacobian product, next to the one-wave visits on the same state."""
import numpy as np
import pytest

import oracle
from synthetic.fields import make_problem
from tests.gpu_common import rel_l2, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("cfg,seed,nx,ny,th,cycles", [
    ("c1", 0, None, None, 64, 1), ("c2", 1, 70, 201, 32, 1), ("c2", 2, 257, 130, 64, 2),
    ("c3", 3, 300, 260, 64, 1), ("c3", 4, 129, 333, 32, 2)])
def test_four_wave_adjoint_fp64(cfg, seed, nx, ny, th, cycles):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem(cfg, seed, nx=nx, ny=ny)
    say(f"[adjoint waves] {cfg} seed={seed} {p.nx}x{p.ny} th={th} cycles={cycles}")
    M, om, src, st = to_dev(p, torch.float64)
    T, par, _, _ = E.solve(M, om, src, p.h, src_t=st, tol=0.0, levels=False)
    To, _, _ = oracle.forward(p)
    po, _ = oracle.parents_levels(p, To)
    assert np.array_equal(par.cpu().numpy(), po)
    g = np.random.default_rng(seed).uniform(-1, 1, To.shape)
    dMo, domo, dso = oracle.vjp(p, To, po, g)
    gd = torch.tensor(g, device=M.device)
    out = {}
    for waves in (1, 4):
        sa = []
        tn = E.tuning(tile_height=th, adjoint_cycles=cycles, adjoint_waves=waves)
        dM, dom, ds = E.adjoint(M, om, T, par, None, src, p.h, gd, src_t=st, tune=tn, stats_out=sa)
        out[waves] = (dM, dom, ds)
        r = rel_l2([dM.cpu().numpy(), dom.cpu().numpy(), ds.cpu().numpy()], [dMo, domo, dso])
        say(f"  waves {waves}: rel L2 {r:.2e}, rounds {sa[0].rounds}")
        assert r <= 1e-10
    # both visits relax to the same fixed point of the same per-node formula
    for a, b in zip(out[1], out[4]):
        assert torch.equal(a, b)


def test_four_wave_adjoint_fp32_and_mixed():
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c2", 5, nx=400, ny=300)
    q = p.rounded(np.float32)
    say("[adjoint waves] 400x300 FP32 and mixed")
    To, _, _ = oracle.forward(q)
    po, _ = oracle.parents_levels(q, To)
    g = np.random.default_rng(1).uniform(0, 1, To.shape)
    dMo, domo, dso = oracle.vjp(q, To, po, g)
    M, om, src, st = to_dev(q, torch.float64)
    T, par, _, _ = E.solve_mixed(M, om, src, p.h, tol=0.0, tol32=1e-5, levels=False)
    assert np.array_equal(par.cpu().numpy(), po)
    for waves in (1, 4):
        dM, dom, ds = E.adjoint_mixed(M, om, T, par, src, p.h, torch.tensor(g, device=M.device),
                                      tune=E.tuning(adjoint_waves=waves))
        r = rel_l2([dM.cpu().numpy(), dom.cpu().numpy(), ds.cpu().numpy()], [dMo, domo, dso])
        say(f"  mixed, waves {waves}: rel L2 {r:.2e}")
        assert r <= 1e-5
