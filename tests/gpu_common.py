"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(p, dtype):
    import torch
    dev = torch.device("cuda:0")
    M = torch.tensor(p.M, dtype=dtype, device=dev).contiguous()
    om = torch.tensor(p.omega, dtype=dtype, device=dev).contiguous()
    src = torch.tensor(p.src_idx, dtype=torch.int32, device=dev)
    st = torch.tensor(p.src_t, dtype=dtype, device=dev)
    return M, om, src, st


def oracle_view(p, dtype):
    """The inputs exactly as a run in ``dtype`` sees them, in float64."""
    return p.rounded(np.float32) if dtype == "f32" else p


def rel_err_cells(Tg, To, skip):
    """max over reached, non-source nodes of |Tg - To| / |To|."""
    m = np.isfinite(To)
    m.flat[skip] = False
    assert np.array_equal(np.isfinite(Tg), np.isfinite(To)), "reached sets differ"
    if not m.any():
        return 0.0
    return float(np.max(np.abs(Tg[m] - To[m]) / np.abs(To[m])))


def check_levels_consistent(parent, level, T):
    """level = 0 at sources, 1 + max over donors elsewhere, -1 unreached; donors strictly earlier in T."""
    ny, nx = parent.shape
    P = parent.astype(np.int64)
    Lv = level.astype(np.int64)
    jj, ii = np.mgrid[0:ny, 0:nx]
    src = P == oracle.SOURCE
    unr = P == oracle.UNREACHED
    assert np.all(Lv[src] == 0)
    assert np.all(Lv[unr] == -1)
    act = ~(src | unr)
    want = np.full(P.shape, -10**9)
    for code in range(16):
        sel = act & (P == code)
        if not sel.any():
            continue
        ks = [code, (code + 1) % 8] if code < 8 else [code - 8]
        best = np.full(sel.sum(), -1)
        for k in ks:
            a, b = ii[sel] + oracle.NBX[k], jj[sel] + oracle.NBY[k]
            assert np.all((a >= 0) & (a < nx) & (b >= 0) & (b < ny))
            assert np.all(T[b, a] < T[sel])
            best = np.maximum(best, Lv[b, a])
        want[sel] = best + 1
    assert np.array_equal(Lv[act], want[act])


def loss_grad_cells(T, cells, target):
    g = np.zeros_like(T)
    g.flat[cells] = 2.0 * (T.flat[cells] - target.flat[cells]) / max(1, len(cells))
    return g


def rel_l2(a, b):
    a = np.concatenate([x.ravel() for x in a])
    b = np.concatenate([x.ravel() for x in b])
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def check_parent_choices(q, To, po, pg, rtol):
    """Where the GPU picked another active update than the oracle, that update
    must reach the oracle's minimum within rtol (a near-tie between candidates:
    either choice is a correct minimiser). Returns the number of such nodes."""
    bad = np.flatnonzero(pg.ravel() != po.ravel())
    for c in bad:
        code = int(pg.flat[c])
        assert code < 16, f"node {c}: GPU code {code} vs oracle {po.flat[c]}"
        v, _ = oracle.candidate(q, To, c, code)
        assert abs(v - To.flat[c]) <= rtol * abs(To.flat[c]), (c, code, int(po.flat[c]), v, To.flat[c])
    return int(bad.size)
