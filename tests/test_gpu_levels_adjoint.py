"""The level-scheduled adjoint (Alg. backward's back-substitution, nodes
counting-sorted by dependency level and solved level by level from the
largest) through the C ABI: against the oracle's VJP, and against the tile
relaxation, which sums the same terms in the same order (equal to the last
bit). Also the forward's levels computed after the concurrent-direction
sweeps (level rounds alone) against the oracle's levels."""
import numpy as np
import pytest

import oracle
from synthetic.fields import make_problem
from tests.gpu_common import FP32_GRAD_RTOL, rel_err_cells, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def tunes(th=64):
    from paper_2603_00035_amd import eikonal as E
    relax = E.tuning(tile_height=th, level_mode=E.LEVELS_AFTER, adjoint_mode=E.ADJ_RELAX)
    lev = E.tuning(tile_height=th, level_mode=E.LEVELS_AFTER, adjoint_mode=E.ADJ_LEVELS)
    return relax, lev


def np64(*xs):
    return [x.double().cpu().numpy() for x in xs]


CASES = [("c1", 0, None, None, 64), ("c2", 1, 70, 201, 32), ("c3", 3, 300, 260, 64), ("c2", 5, 257, 130, 64),
         ("c1", 2, 1, 70, 64), ("c1", 4, 70, 1, 32)]


@pytest.mark.parametrize("cfg,seed,nx,ny,th", CASES)
def test_levels_after_and_level_adjoint_fp64(cfg, seed, nx, ny, th):
    from paper_2603_00035_amd import eikonal as E
    p = make_problem(cfg, seed, nx=nx, ny=ny)
    say(f"[levels fp64] {cfg} seed={seed} {p.nx}x{p.ny} th={th}")
    M, om, src, st = to_dev(p, torch.float64)
    relax, lev_t = tunes(th)
    T, par, lev, s = E.solve(M, om, src, p.h, src_t=st, tol=0.0, tune=relax, levels=True)
    assert s.converged
    To, _, _ = oracle.forward(p)
    po, lo = oracle.parents_levels(p, To)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    assert np.array_equal(par.cpu().numpy(), po)
    assert np.array_equal(lev.cpu().numpy(), lo)
    g = np.random.default_rng(seed).uniform(-1, 1, To.shape)
    gT = torch.tensor(g, device=M.device)
    r_rel = E.adjoint(M, om, T, par, None, src, p.h, gT, src_t=st, tune=relax)
    r_lev = E.adjoint(M, om, T, par, lev, src, p.h, gT, src_t=st, tune=lev_t)
    for a, b in zip(np64(*r_rel), np64(*r_lev)):
        assert np.array_equal(a, b)
    dMo, domo, dso = oracle.vjp(p, To, po, g)
    assert rel_l2(np64(*r_lev), [dMo, domo, dso]) <= 1e-10


def test_level_adjoint_fp32_c2_loss():
    from paper_2603_00035_amd import eikonal as E
    from tests.gpu_common import loss_grad_cells
    from synthetic.fields import Problem
    p = make_problem("c2", 0)
    q = p.rounded(np.float32)
    say("[levels fp32] c2 512x512 tol 1e-5, 256 loss cells")
    M, om, src, _ = to_dev(p, torch.float32)
    relax, lev_t = tunes()
    T, par, lev, s = E.solve(M, om, src, p.h, tol=1e-5, tune=relax, levels=True)
    assert s.converged
    To, _, _ = oracle.forward(q)
    po, _ = oracle.parents_levels(q, To)
    tgt = make_problem("c2", 1).rounded(np.float32)
    Tt, _, _ = oracle.forward(Problem(q.nx, q.ny, q.h, tgt.M, tgt.omega, q.src_idx, q.src_t))
    Tg = T.double().cpu().numpy()
    gT = torch.tensor(loss_grad_cells(Tg, p.loss_idx, Tt), dtype=torch.float32, device=M.device)
    r_rel = np64(*E.adjoint(M, om, T, par, None, src, p.h, gT, tune=relax))
    r_lev = np64(*E.adjoint(M, om, T, par, lev, src, p.h, gT, tune=lev_t))
    for a, b in zip(r_rel, r_lev):
        assert np.array_equal(a, b)
    dMo, domo, _ = oracle.vjp(q, To, po, loss_grad_cells(To, p.loss_idx, Tt))
    r = rel_l2(r_lev[:2], [dMo, domo])
    say(f"  gradient rel L2 {r:.2e}")
    assert r <= FP32_GRAD_RTOL


def test_level_adjoint_mixed_stress():
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c3", 7, nx=320, ny=288)
    say("[levels mixed] 320x288 stress recipe, tol 0")
    M, om, src, _ = to_dev(p, torch.float64)
    relax, lev_t = tunes()
    T, par, lev, (s32, s64) = E.solve_mixed(M, om, src, p.h, tol=0.0, tol32=1e-5, tune32=relax, tune=relax,
                                            levels=True)
    assert s64.converged
    To, _, _ = oracle.forward(p)
    po, lo = oracle.parents_levels(p, To)
    assert rel_err_cells(T.cpu().numpy(), To, p.src_idx) <= 1e-12
    assert np.array_equal(lev.cpu().numpy(), lo)
    g = np.random.default_rng(1).uniform(0, 1, To.shape)
    gT = torch.tensor(g, device=M.device)
    r_rel = np64(*E.adjoint_mixed(M, om, T, par, src, p.h, gT, tune=relax))
    r_lev = np64(*E.adjoint_mixed(M, om, T, par, src, p.h, gT, tune=lev_t, level=lev))
    for a, b in zip(r_rel, r_lev):
        assert np.array_equal(a, b)
    dMo, domo, dso = oracle.vjp(p, To, po, g)
    assert rel_l2(r_lev, [dMo, domo, dso]) <= 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_level_adjoint_batched(dtype):
    from paper_2603_00035_amd import eikonal as E
    from tests.test_gpu_batched import SIZES, make_batch, packed_inputs, uneven_set
    dt = torch.float64 if dtype == "f64" else torch.float32
    probs = uneven_set(len(SIZES), 700, SIZES)
    say(f"[levels batched {dtype}] {len(probs)} grids")
    relax, lev_t = tunes()
    B = make_batch(probs, dt, tune=lev_t)
    M, om, src = packed_inputs(B, probs, dt)
    T, par, lev, st = B.forward(M, om, src, tol=0.0, levels=True)
    assert st.converged
    gs = [np.random.default_rng(g).uniform(-1, 1, (p.ny, p.nx)) for g, p in enumerate(probs)]
    gT = torch.tensor(np.concatenate([x.ravel() for x in gs]), dtype=dt, device=B.device)
    dM, dom, ds, _ = B.backward(M, om, T, par, lev, src, gT)
    B2 = make_batch(probs, dt, tune=relax)
    dM2, dom2, ds2, _ = B2.backward(M, om, T, par, None, src, gT)
    for a, b in zip(np64(dM, dom, ds), np64(dM2, dom2, ds2)):
        assert np.array_equal(a, b)
    if dtype == "f32":
        return
    dMs, doms = B.unpack_planes(dM, 3), B.unpack_planes(dom, 2)
    for g, p in enumerate(probs):
        To, _, _ = oracle.forward(p)
        po, _ = oracle.parents_levels(p, To)
        dMo, domo, dso = oracle.vjp(p, To, po, gs[g])
        dsg = ds[B.src_offsets[g]:B.src_offsets[g + 1]].cpu().numpy()
        assert rel_l2([dMs[g].cpu().numpy(), doms[g].cpu().numpy(), dsg], [dMo, domo, dso]) <= 1e-10, g


def test_level_adjoint_requires_levels():
    from paper_2603_00035_amd import _lib as L
    from paper_2603_00035_amd import eikonal as E
    p = make_problem("c1", 0, nx=40, ny=30)
    M, om, src, _ = to_dev(p, torch.float64)
    T, par, _, _ = E.solve(M, om, src, p.h, tol=0.0, levels=False)
    _, lev_t = tunes()
    with pytest.raises(L.EikError) as ei:
        E.adjoint(M, om, T, par, None, src, p.h, torch.ones_like(T), tune=lev_t)
    assert ei.value.code == L.EIK_EINVAL
