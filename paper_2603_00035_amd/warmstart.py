"""Learned warm start: training set from the batched GPU solver, training with
the network's own kernels, and the warm-vs-cold evaluation with fallback.

Usage (on the GPU): python -m paper_2603_00035_amd.warmstart --train 20000 --eval 1000 --out DIR
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import eikonal as E
from .batched import Batch
from .unet import UNet

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "unet_warmstart_256.pt")


def _pack_sources(src):
    """src (B, max_src) with -1 padding -> (counts, packed int32 tensor)."""
    valid = src >= 0
    counts = valid.sum(dim=1).tolist()
    return counts, src[valid].contiguous()


def solve_batch(M, om, src, h, tol=1e-5, T_init=None, max_rounds=256, tune=None, fallback=False):
    """Equal-size grids M (B,3,ny,nx), omega (B,2,ny,nx), sources (B,max_src).
    Returns T (B,ny,nx), parent (B,ny,nx), Stats, seconds (synchronised).
    ``fallback``: the library's residual monitor (EIK_WARM_FALLBACK) drops a
    warm start that leaves more than a quarter of the tiles changing after two
    rounds and solves from the cold start."""
    B, _, ny, nx = M.shape
    counts, packed = _pack_sources(src)
    batch = Batch([(nx, ny, h, c) for c in counts], dtype=M.dtype, device=M.device, tune=tune,
                  max_rounds=max_rounds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T, par, _, st = batch.forward(M.reshape(-1), om.reshape(-1), packed,
                                  T_init=None if T_init is None else T_init.reshape(-1), tol=tol,
                                  warm_fallback=fallback)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return T.reshape(B, ny, nx), par.reshape(B, ny, nx), st, dt


def make_training_set(n, seed0=0, chunk=256, device="cuda"):
    from synthetic.fields_torch import random_batch
    Ms, oms, srcs, Ts = [], [], [], []
    h = None
    for k in range(0, n, chunk):
        b = min(chunk, n - k)
        M, om, src, h = random_batch(seed0 + k, b, device=device)
        T, _, st, _ = solve_batch(M, om, src, h)
        assert st.converged
        Ms.append(M)
        oms.append(om)
        srcs.append(src)
        Ts.append(T)
    return torch.cat(Ms), torch.cat(oms), torch.cat(srcs), h, torch.cat(Ts)


def targets(net, M, om, src, h, T):
    """Fills the network input buffer; returns the target ratio T / (d + h)."""
    B = M.shape[0]
    hv = torch.full((B,), h, dtype=torch.float32, device=M.device)
    d = net.features(M, om, src, hv)
    return (T / (d + h)).reshape(-1).contiguous(), d


def train(net, data, epochs=4, batch=32, lr=1e-3, log=print):
    M, om, src, h, T = data
    n = M.shape[0]
    g = torch.Generator(device=M.device).manual_seed(1)
    steps = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=M.device)
        losses = []
        lr_ep = lr if ep < epochs - 1 else lr * 0.3
        t0 = time.perf_counter()
        for k in range(0, n - batch + 1, batch):
            idx = perm[k:k + batch]
            tgt, _ = targets(net, M[idx].contiguous(), om[idx].contiguous(), src[idx].contiguous(), h, T[idx])
            losses.append(net.train_step(tgt, lr=lr_ep))
            steps += 1
        torch.cuda.synchronize()
        mean = float(torch.cat(losses).mean())
        log(f"epoch {ep}: mean loss {mean:.3e} over {len(losses)} steps, {time.perf_counter() - t0:.1f} s")
    return steps


def predict(net, M, om, src, h):
    B, _, ny, nx = M.shape
    hv = torch.full((B,), h, dtype=torch.float32, device=M.device)
    d = net.features(M, om, src, hv)
    r = net.forward(B, ny, nx).reshape(B, ny, nx)
    return r * (d + h)


def evaluate(net, seeds, chunk=250, tol=1e-5, log=print):
    """Warm vs cold on held-out seeds of the numpy generator, batched.

    cold: the cold-start solve. warm: inference + the solve from the network's
    field, run to convergence (its sweeps, time and distance to the cold
    result). warm_fb: the deployable policy -- inference + the solve with the
    library's residual monitor, which drops the warm field after two
    full-update rounds when more than a quarter of the tiles are still
    changing and solves from the cold start (both charged)."""
    from synthetic.fields import make_problem
    dev = torch.device("cuda")
    res = {"grids": 0, "cold_s": 0.0, "warm_s": 0.0, "warm_fb_s": 0.0, "infer_s": 0.0, "cold_updates": 0,
           "warm_updates": 0, "cold_rounds": [], "warm_rounds": [], "fb_rounds": [], "fallback_batches": 0,
           "batches": 0, "max_rel_fb_vs_cold": 0.0,
           "max_rel_warm_vs_cold": 0.0, "pred_rel_err_mean": [], "pred_rel_err_p99": []}
    for k in range(0, len(seeds), chunk):
        ps = [make_problem("c5", int(s)) for s in seeds[k:k + chunk]]
        B = len(ps)
        M = torch.tensor(np.stack([p.M for p in ps]), dtype=torch.float32, device=dev)
        om = torch.tensor(np.stack([p.omega for p in ps]), dtype=torch.float32, device=dev)
        src = torch.full((B, 4), -1, dtype=torch.int32)
        for b, p in enumerate(ps):
            src[b, :p.src_idx.size] = torch.tensor(p.src_idx)
        src = src.to(dev)
        h = ps[0].h
        ny, nx = M.shape[2], M.shape[3]
        Tc, _, stc, tc = solve_batch(M, om, src, h, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Tinit = predict(net, M, om, src, h)
        torch.cuda.synchronize()
        ti = time.perf_counter() - t0
        m = torch.isfinite(Tc) & (Tc > 0)
        perr = ((Tinit - Tc).abs()[m] / Tc[m]).float()
        Tw, _, stw, tw = solve_batch(M, om, src, h, tol=tol, T_init=Tinit, max_rounds=4096)
        Tb, _, stb, tb = solve_batch(M, om, src, h, tol=tol, T_init=Tinit, max_rounds=4096, fallback=True)
        assert stb.converged
        t_fb = ti + tb
        res["fallback_batches"] += int(stb.fell_back)
        res["fb_rounds"].append(stb.rounds)
        res["max_rel_fb_vs_cold"] = max(res["max_rel_fb_vs_cold"], ((Tb - Tc).abs()[m] / Tc[m]).max().item())
        rel = ((Tw - Tc).abs()[m] / Tc[m]).max().item()
        res["grids"] += B
        res["batches"] += 1
        res["cold_s"] += tc
        res["warm_s"] += tw + ti
        res["warm_fb_s"] += t_fb
        res["infer_s"] += ti
        res["cold_updates"] += stc.cell_updates
        res["warm_updates"] += stw.cell_updates
        res["cold_rounds"].append(stc.rounds)
        res["warm_rounds"].append(stw.rounds)
        res["max_rel_warm_vs_cold"] = max(res["max_rel_warm_vs_cold"], rel)
        res["pred_rel_err_mean"].append(perr.mean().item())
        res["pred_rel_err_p99"].append(torch.quantile(perr[:1 << 24], 0.99).item())
        log(f"eval {k + B}/{len(seeds)}: cold {tc * 1e3:.1f} ms ({stc.rounds} rounds, "
            f"{stc.cell_updates / (B * nx * ny):.1f} sweeps/node); warm {tw * 1e3:.1f} ms + inference {ti * 1e3:.1f} ms "
            f"({stw.rounds} rounds, {stw.cell_updates / (B * nx * ny):.1f} sweeps/node); prediction rel err mean "
            f"{perr.mean().item():.2e}; warm vs cold max rel diff {rel:.2e}")
    n_cells = res["grids"] * 256 * 256
    res["cold_sweeps_per_node"] = res["cold_updates"] / n_cells
    res["warm_sweeps_per_node"] = res["warm_updates"] / n_cells
    res["speedup_warm"] = res["cold_s"] / res["warm_s"]
    res["speedup_warm_with_fallback"] = res["cold_s"] / res["warm_fb_s"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=20000)
    ap.add_argument("--eval", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default="gpurun_out/warmstart")
    ap.add_argument("--load", default=None, help="skip training, load these weights")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    logf = open(os.path.join(args.out, "log.txt"), "w")

    def log(s):
        print(s, flush=True)
        logf.write(s + "\n")
        logf.flush()

    net = UNet()
    report = {}
    if args.load:
        net.load_state_dict(torch.load(args.load, weights_only=True))
    else:
        t0 = time.perf_counter()
        data = make_training_set(args.train)
        torch.cuda.synchronize()
        log(f"training set: {args.train} solves in {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        report["train_steps"] = train(net, data, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
        report["train_s"] = time.perf_counter() - t0
        del data
        torch.save(net.state_dict(), os.path.join(args.out, "unet_warmstart_256.pt"))
    seeds = list(range(1_000_000, 1_000_000 + args.eval))
    report.update(evaluate(net, seeds, log=log))
    log(json.dumps({k: v for k, v in report.items() if not isinstance(v, list)}))
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
