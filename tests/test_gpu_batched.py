"""Batched solving of uneven grids through the C ABI, against the oracle grid by
grid, against single-grid solves, and replayed from a captured HIP graph."""
import numpy as np
import pytest

import oracle
from synthetic.fields import Problem, make_problem
from tests.gpu_common import check_parent_choices, rel_err_cells, rel_l2, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def uneven_set(n, seed0, sizes=None):
    probs = []
    rng = np.random.default_rng(seed0)
    for g in range(n):
        if sizes is not None:
            nx, ny = sizes[g % len(sizes)]
        else:
            nx, ny = int(rng.integers(20, 160)), int(rng.integers(20, 160))
        probs.append(make_problem("c4", seed0 + g, nx=nx, ny=ny))
    return probs


def packed_inputs(B, probs, dtype):
    dev = B.device
    M, om = B.pack([torch.tensor(p.M) for p in probs], [torch.tensor(p.omega) for p in probs])
    src = torch.tensor(np.concatenate([p.src_idx for p in probs]), dtype=torch.int32, device=dev)
    return M, om, src


def make_batch(probs, dtype, **kw):
    from paper_2603_00035_amd.batched import Batch
    return Batch([(p.nx, p.ny, p.h, p.src_idx.size) for p in probs], dtype=dtype, **kw)


SIZES = [(1, 5), (70, 3), (64, 64), (65, 33), (130, 97), (7, 200), (128, 128), (33, 65), (200, 7), (97, 130)]


@pytest.mark.parametrize("th", [64, 32])
def test_batched_fp64_matches_oracle_per_grid(th):
    from paper_2603_00035_amd import eikonal as E
    probs = uneven_set(len(SIZES), 500, SIZES)
    say(f"[batched fp64] {len(probs)} grids, tile height {th}")
    B = make_batch(probs, torch.float64, tune=E.tuning(tile_height=th))
    M, om, src = packed_inputs(B, probs, torch.float64)
    T, par, lev, st = B.forward(M, om, src, tol=0.0, levels=True)
    assert st.converged
    Ts, ps, ls = B.unpack_nodes(T), B.unpack_nodes(par), B.unpack_nodes(lev)
    gs = []
    for g, p in enumerate(probs):
        To, _, _ = oracle.forward(p)
        po, lo = oracle.parents_levels(p, To)
        Tg = Ts[g].cpu().numpy()
        assert rel_err_cells(Tg, To, p.src_idx) <= 1e-12, g
        assert np.array_equal(ps[g].cpu().numpy(), po), g
        assert np.array_equal(ls[g].cpu().numpy(), lo), g
        gs.append(np.random.default_rng(g).uniform(-1, 1, To.shape))
    gT = torch.tensor(np.concatenate([x.ravel() for x in gs]), dtype=torch.float64, device=B.device)
    dM, dom, ds, rounds = B.backward(M, om, T, par, None, src, gT)  # the adjoint needs no levels
    dMs, doms = B.unpack_planes(dM, 3), B.unpack_planes(dom, 2)
    for g, p in enumerate(probs):
        To, _, _ = oracle.forward(p)
        po, _ = oracle.parents_levels(p, To)
        dMo, domo, dso = oracle.vjp(p, To, po, gs[g])
        dsg = ds[B.src_offsets[g]:B.src_offsets[g + 1]].cpu().numpy()
        assert rel_l2([dMs[g].cpu().numpy(), doms[g].cpu().numpy(), dsg], [dMo, domo, dso]) <= 1e-10, g


def test_batched_fp32_matches_oracle_and_single_solves():
    from paper_2603_00035_amd import eikonal as E
    probs = uneven_set(12, 900)
    say(f"[batched fp32] {len(probs)} random grids")
    B = make_batch(probs, torch.float32)
    M, om, src = packed_inputs(B, probs, torch.float32)
    T, par, lev, st = B.forward(M, om, src, tol=0.0)
    Ts = B.unpack_nodes(T)
    for g, p in enumerate(probs):
        q = p.rounded(np.float32)
        To, _, _ = oracle.forward(q)
        Tg = Ts[g].double().cpu().numpy()
        assert rel_err_cells(Tg, To, p.src_idx) <= 1e-5, g
        # the single-grid solve with the same kernels, tiling and knobs reaches
        # the same FP32 fixed point up to the last bits (the concurrent-direction
        # cold start can settle rounding-level ties in either order)
        dev = B.device
        Ti, pi, li, _ = E.solve(torch.tensor(p.M, dtype=torch.float32, device=dev),
                                torch.tensor(p.omega, dtype=torch.float32, device=dev),
                                torch.tensor(p.src_idx, device=dev), p.h, tol=0.0, tune=B.tune, levels=False)
        a, b = Ti.reshape(-1).double(), Ts[g].reshape(-1).double()
        fin = torch.isfinite(b)
        assert torch.equal(torch.isfinite(a), fin), g
        assert bool(((a[fin] - b[fin]).abs() <= 4 * 2.0 ** -23 * b[fin].abs()).all()), g
        po, _ = oracle.parents_levels(q, To)
        check_parent_choices(q, To, po, B.unpack_nodes(par)[g].cpu().numpy(), 1e-5)


def test_graph_capture_replays_match_eager():
    """The unsynchronised batched forward + backward captured once in a HIP
    graph and replayed three times on changed inputs, with eager work between
    the replays; every replay equals the eager (synchronised) result bit for
    bit. The solves run to exact stationarity: at a positive tolerance the
    concurrent-direction visits fix the field only to within that tolerance
    (which store of a sub-tolerance change lands last depends on timing)."""
    probs = uneven_set(16, 1300)
    say(f"[graph] {len(probs)} grids")
    B = make_batch(probs, torch.float32, max_rounds=256)
    M, om, src = packed_inputs(B, probs, torch.float32)
    Ms, oms = M.clone(), om.clone()
    gT = torch.rand(B.n_nodes, device=B.device)
    fo = B.alloc_forward()
    bo = B.alloc_backward()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture
        B.forward(Ms, oms, src, tol=0.0, out=fo, sync=False)
        B.backward(Ms, oms, fo[0], fo[1], fo[2], src, gT, out=bo, sync=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.forward(Ms, oms, src, tol=0.0, out=fo, sync=False)
        B.backward(Ms, oms, fo[0], fo[1], fo[2], src, gT, out=bo, sync=False)
    torch.cuda.synchronize()
    for rep in range(3):
        scale = 1.0 + 0.1 * rep
        Ms.copy_(M * scale * scale)  # T scales by `scale` under (a^2 M, a omega)
        oms.copy_(om * scale)
        graph.replay()
        torch.cuda.synchronize()
        assert B.pending() == (0, 0, 0)
        Tr, dMr = fo[0].clone(), bo[0].clone()
        x = torch.randn(1000, device=B.device).sum()  # eager work between replays
        Te, pe, le, st = B.forward(Ms, oms, src, tol=0.0)
        dMe, dome, dse, _ = B.backward(Ms, oms, Te, pe, le, src, gT)
        torch.cuda.synchronize()
        assert torch.isfinite(x)
        assert torch.equal(Tr, Te), rep
        assert torch.equal(dMr, dMe), rep


def test_batched_mixed_degenerate_grids_match_oracle():
    """The mixed-precision batch (FP32 sweeps, FP64 sweeps to exact
    stationarity, mixed adjoint) on degenerate grids packed beside ordinary
    ones: a single node, single rows and columns, a 2 x 2 grid, grids one node
    wider or taller than a tile."""
    from synthetic.fields import constant_problem
    sizes = [(1, 70), (70, 1), (2, 2), (65, 1), (1, 65), (64, 64), (65, 33), (3, 129)]
    probs = [constant_problem(1, 1, 0.1, 1.3, 0.2, 0.7, 0.1, -0.05, [(0, 0)])] + uneven_set(len(sizes), 1300, sizes)
    say(f"[batched mixed] {len(probs)} degenerate and ordinary grids")
    B = make_batch(probs, torch.float64, mixed=True)
    M, om, src = packed_inputs(B, probs, torch.float64)
    T, par, _, st = B.forward(M, om, src, tol=0.0, tol32=1e-5, tol64=0.0)
    assert st.converged
    Ts, ps = B.unpack_nodes(T), B.unpack_nodes(par)
    gs = [np.random.default_rng(g).uniform(0, 1, (p.ny, p.nx)) for g, p in enumerate(probs)]
    gT = torch.tensor(np.concatenate([x.ravel() for x in gs]), dtype=torch.float64, device=B.device)
    dM, dom, ds, _ = B.backward(M, om, T, par, None, src, gT)
    dMs, doms = B.unpack_planes(dM, 3), B.unpack_planes(dom, 2)
    for g, p in enumerate(probs):
        To, _, _ = oracle.forward(p)
        po, _ = oracle.parents_levels(p, To)
        assert rel_err_cells(Ts[g].cpu().numpy(), To, p.src_idx) <= 1e-12, g
        assert np.array_equal(ps[g].cpu().numpy(), po), g
        dMo, domo, dso = oracle.vjp(p, To, po, gs[g])
        dsg = ds[B.src_offsets[g]:B.src_offsets[g + 1]].cpu().numpy()
        # FP64 weights, FP32 relaxation of lambda
        assert rel_l2([dMs[g].cpu().numpy(), doms[g].cpu().numpy(), dsg], [dMo, domo, dso]) <= 1e-5, g
