"""Autotuner for the solver's scheduling knobs.

The knobs (tile height, local sweep cycles per round, rounds between host
convergence checks, the optional fast cold-start phase, adjoint and level
round budgets) change only how the work is scheduled, never the fixed point
that is computed. Their best values depend on the grid size, the dtype and the
medium, so they are chosen by timing per size class on synthetic problems of
that class and stored in a small JSON table next to this module; ``lookup``
returns the entry for a grid and the solve calls use it when the caller passes
no tuning of its own.

Tuning is a coordinate descent from the library defaults: each knob in turn
takes every candidate value with the others held, and the fastest
forward + adjoint time (median of a few repeats) is kept.

Usage (on the GPU): python -m paper_2603_00035_amd.autotune --out paper_2603_00035_amd/tuning_table.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import _lib as L

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning_table.json")
KNOBS = ("tile_height", "max_local_cycles", "rounds_per_check", "fast_cold_start", "adjoint_rounds", "level_rounds",
         "scheduler", "node_lanes", "adjoint_cycles", "adjoint_waves", "full_waves")
DEFAULTS = {"tile_height": 64, "max_local_cycles": 1, "rounds_per_check": 8, "fast_cold_start": 2,
            "adjoint_rounds": 64, "level_rounds": 8, "scheduler": 1, "node_lanes": 4,
            "adjoint_cycles": 1, "adjoint_waves": 4, "full_waves": 4}
CANDIDATES = {"tile_height": (32, 64), "max_local_cycles": (1, 2, 3), "rounds_per_check": (4, 8, 16, 32),
              "fast_cold_start": (0, 1, 2), "adjoint_rounds": (16, 64, 256), "level_rounds": (4, 8, 16),
              "scheduler": (1, 2), "node_lanes": (1, 2, 4), "adjoint_cycles": (1, 2),
              "adjoint_waves": (1, 4), "full_waves": (1, 4)}
# knobs timed by the tuner (the unsynchronised round budgets are sized for
# correctness, not speed, and keep their defaults)
TUNED = ("tile_height", "max_local_cycles", "rounds_per_check", "fast_cold_start", "scheduler", "node_lanes",
         "adjoint_cycles", "adjoint_waves", "full_waves")
# single-grid size classes by node count: (upper bound, representative side, problem recipe)
CLASSES = ((96 * 96, 64, "c1"), (384 * 384, 256, "c1"), (768 * 768, 512, "c2"), (1536 * 1536, 1024, "c3"),
           (1 << 62, 2048, "c3"))
# batch classes by total node count: (upper bound, grids in the representative batch)
BATCH_CLASSES = ((8 << 20, 64), (1 << 62, 256))

_cache = {}


def _load(path=TABLE):
    if path not in _cache:
        try:
            with open(path) as f:
                _cache[path] = json.load(f)
        except (OSError, ValueError):
            _cache[path] = None
    return _cache[path]


def lookup(n_nodes, dtype_name, kind="single", path=TABLE):
    """EikTuning for a grid (kind "single") or a batch (kind "batch") of
    ``n_nodes`` nodes in dtype "f32"/"f64", or None when the table is absent or
    has no entry for that dtype and kind."""
    table = _load(path)
    if not table:
        return None
    best = None
    for e in table.get("entries", []):
        if e["dtype"] != dtype_name or e.get("kind", "single") != kind:
            continue
        if n_nodes <= e["max_nodes"] and (best is None or e["max_nodes"] < best["max_nodes"]):
            best = e
    if best is None:
        return None
    t = best["tuning"]
    return L.EikTuning(*[int(t[k]) for k in KNOBS])


def dtype_name(dtype):
    import torch
    return {torch.float32: "f32", torch.float64: "f64"}[dtype]


# -- timing ---------------------------------------------------------------
def _problem(recipe, side, seed, dtype):
    import torch
    from synthetic.fields import make_problem
    p = make_problem(recipe, seed, nx=side, ny=side)
    dev = torch.device("cuda")
    M = torch.tensor(p.M, dtype=dtype, device=dev)
    om = torch.tensor(p.omega, dtype=dtype, device=dev)
    src = torch.tensor(p.src_idx, dtype=torch.int32, device=dev)
    g = torch.rand(side, side, generator=torch.Generator(device=dev).manual_seed(seed), device=dev, dtype=dtype)
    return M, om, src, p.h, g


def _batch_problem(n_grids, seed0, dtype):
    import numpy as np
    import torch
    from synthetic.fields import batched_set
    probs = batched_set(n_grids, seed0)
    dev = torch.device("cuda")
    cat = lambda xs: torch.tensor(np.concatenate([x.reshape(-1) for x in xs]), dtype=dtype, device=dev)
    M, om = cat([p.M for p in probs]), cat([p.omega for p in probs])
    src = torch.tensor(np.concatenate([p.src_idx for p in probs]), dtype=torch.int32, device=dev)
    shapes = [(p.nx, p.ny, p.h, p.src_idx.size) for p in probs]
    g = torch.rand(M.numel() // 3, generator=torch.Generator(device=dev).manual_seed(seed0), device=dev, dtype=dtype)
    return ("batch", shapes, M, om, src, g)


def time_batch(prob, knobs, tol, reps=3):
    """Median wall time (ms) of one batched forward + adjoint with these knobs."""
    import torch
    from .batched import Batch
    _, shapes, M, om, src, g = prob
    tn = L.EikTuning(*[int(knobs[k]) for k in KNOBS])
    B = Batch(shapes, dtype=M.dtype, device=M.device, tune=tn, max_rounds=4096)
    times = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, par, _, st = B.forward(M, om, src, tol=tol)
        B.backward(M, om, T, par, None, src, g)
        torch.cuda.synchronize()
        if r:
            times.append(1e3 * (time.perf_counter() - t0))
        if not st.converged:
            return float("inf")
    times.sort()
    return times[len(times) // 2]


def time_fwd_adj(prob, knobs, tol, reps=3):
    """Median wall time (ms) of one forward + adjoint with these knobs."""
    import torch
    from . import eikonal as E
    if prob[0] == "batch":
        return time_batch(prob, knobs, tol, reps)
    M, om, src, h, g = prob
    tn = L.EikTuning(*[int(knobs[k]) for k in KNOBS])
    ws = E.workspace(E.make_grid(M.shape[2], M.shape[1], h, src), L.dtype_code(M), M.device)
    times = []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, par, _, st = E.solve(M, om, src, h, tol=tol, tune=tn, ws=ws, levels=False)
        E.adjoint(M, om, T, par, None, src, h, g, tune=tn, ws=ws)
        torch.cuda.synchronize()
        if r:
            times.append(1e3 * (time.perf_counter() - t0))
        if not st.converged:
            return float("inf")
    times.sort()
    return times[len(times) // 2]


def tune_class(prob, tol, passes=2, log=print):
    cur = dict(DEFAULTS)
    base = time_fwd_adj(prob, cur, tol)
    best_t = base
    for _ in range(passes):
        changed = False
        for k in TUNED:
            for v in CANDIDATES[k]:
                if v == cur[k]:
                    continue
                trial = dict(cur, **{k: v})
                t = time_fwd_adj(prob, trial, tol)
                log(f"  {k}={v}: {t:.3f} ms (best {best_t:.3f})")
                if t < 0.97 * best_t:
                    cur, best_t, changed = trial, t, True
        if not changed:
            break
    return cur, best_t, base


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-side", type=int, default=2048)
    args = ap.parse_args()
    entries = []
    for dn in args.dtypes.split(","):
        dtype = {"f32": torch.float32, "f64": torch.float64}[dn]
        for max_nodes, side, recipe in CLASSES:
            if side > args.max_side:
                continue
            prob = _problem(recipe, side, 0, dtype)
            print(f"[tune] {dn} {side}x{side} ({recipe})", flush=True)
            knobs, t, base = tune_class(prob, args.tol)
            print(f"[tune] {dn} {side}x{side}: {base:.3f} ms -> {t:.3f} ms with {knobs}", flush=True)
            entries.append({"kind": "single", "dtype": dn, "max_nodes": max_nodes, "side": side, "recipe": recipe,
                            "tuning": knobs, "ms_fwd_adj": round(t, 4), "ms_default": round(base, 4)})
        if dn == "f32":
            for max_nodes, n_grids in BATCH_CLASSES:
                prob = _batch_problem(n_grids, 1000, dtype)
                print(f"[tune] {dn} batch of {n_grids} grids", flush=True)
                knobs, t, base = tune_class(prob, args.tol)
                print(f"[tune] {dn} batch of {n_grids}: {base:.3f} ms -> {t:.3f} ms with {knobs}", flush=True)
                entries.append({"kind": "batch", "dtype": dn, "max_nodes": max_nodes, "grids": n_grids,
                                "recipe": "c4", "tuning": knobs, "ms_fwd_adj": round(t, 4),
                                "ms_default": round(base, 4)})
    out = {"device": torch.cuda.get_device_name(0), "tol": args.tol, "knobs": list(KNOBS), "entries": entries}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
