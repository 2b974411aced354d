"""The batched workload at its own shape: 256 grids with sides drawn from
64..512 (non-square), ratio-4 metrics, drift 0.5, 1-4 sources each, FP32,
forward to 1e-5 and adjoint captured once in a HIP graph and replayed (fixed
round budgets, no host synchronisation). A fixed sample of 16 grids, the
largest among them, is checked against the oracle run to stationarity on the
same FP32-rounded inputs: forward to 1e-5 at every node, parameter gradient
of a dense linear functional to the FP32 bar (four times the FP32-storage
floor the oracle measures on that grid, or 1e-4 where that is looser)."""
import numpy as np
import pytest

import oracle
from synthetic.fields import batched_set
from tests.gpu_common import FP32_FLOOR_FACTOR, fp32_storage_floor, rel_err_cells, rel_l2, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.timeout(900)
def test_batched_256_uneven_grids_graph_replay():
    from paper_2603_00035_amd.batched import Batch
    probs = batched_set(256, 1000)
    n_cells = sum(p.n for p in probs)
    say(f"[c4 shape] {len(probs)} grids, {n_cells} cells, largest {max(p.n for p in probs)}")
    dev = torch.device("cuda:0")
    q = [p.rounded(np.float32) for p in probs]
    shapes = [(p.nx, p.ny, p.h, p.src_idx.size) for p in probs]
    cat = lambda xs: torch.tensor(np.concatenate([x.reshape(-1) for x in xs]), dtype=torch.float32, device=dev)
    M, om = cat([p.M for p in q]), cat([p.omega for p in q])
    src = torch.tensor(np.concatenate([p.src_idx for p in probs]), dtype=torch.int32, device=dev)
    weights = [np.random.default_rng(50_000 + g).uniform(0, 1, (p.ny, p.nx)) for g, p in enumerate(probs)]
    gT = cat(weights)
    B = Batch(shapes, dtype=torch.float32, device=dev, max_rounds=4096)
    _, _, _, st = B.forward(M, om, src, tol=1e-5)
    assert st.converged
    B.max_rounds = int(st.rounds * 1.25) + 8
    fo, bo = B.alloc_forward(), B.alloc_backward()

    def step():
        B.forward(M, om, src, tol=1e-5, out=fo, sync=False)
        B.backward(M, om, fo[0], fo[1], fo[2], src, gT, out=bo, sync=False)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    fo[0].fill_(0.0)
    graph.replay()
    torch.cuda.synchronize()
    assert B.pending() == (0, 0, 0), "the fixed round budgets ran out"
    Ts, ps = B.unpack_nodes(fo[0]), B.unpack_nodes(fo[1])
    dMs, doms = B.unpack_planes(bo[0], 3), B.unpack_planes(bo[1], 2)
    largest = int(np.argmax([p.n for p in probs]))
    sample = sorted({largest, *np.random.default_rng(3).choice(len(probs), 15, replace=False).tolist()})
    worst_f, worst_g = 0.0, 0.0
    for g in sample:
        qg = q[g]
        To, _, sto = oracle.forward(qg)
        assert sto == 0
        po, _ = oracle.parents_levels(qg, To)
        Tg = Ts[g].double().cpu().numpy()
        err = rel_err_cells(Tg, To, qg.src_idx)
        dMo, domo, _ = oracle.vjp(qg, To, po, weights[g])
        r = rel_l2([dMs[g].double().cpu().numpy(), doms[g].double().cpu().numpy()], [dMo, domo])
        floor = fp32_storage_floor(qg, To, po, lambda T: weights[g])
        say(f"  grid {g} {qg.nx}x{qg.ny}: forward {err:.2e}, gradient {r:.2e} (FP32-storage floor {floor:.2e})")
        assert err <= 1e-5, g
        assert r <= max(1e-4, FP32_FLOOR_FACTOR * floor), g
        worst_f, worst_g = max(worst_f, err), max(worst_g, r)
    say(f"  worst over the sample: forward {worst_f:.2e}, gradient {worst_g:.2e}")
