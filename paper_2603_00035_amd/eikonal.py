"""PyTorch-facing API of the gfx950 Randers eikonal library.

``solve`` / ``adjoint`` call ``eik_forward`` / ``eik_backward``; ``EikonalFn``
wraps them as a ``torch.autograd.Function`` (implicit differentiation of the
converged fixed point, Sec. 3.3); ``ProjectFn`` wraps ``eik_project`` and its
VJP (App. learning details). PyTorch provides device memory and the stream;
the arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L
from . import autotune


@dataclass
class Stats:
    rounds: int
    converged: bool
    cell_updates: int
    n_levels: int
    status: int
    sweep_launches: int = 0
    sweep_ms: float = 0.0
    aux_rounds: int = 0
    fast_ms: float = 0.0
    fast_cell_updates: int = 0
    fast_launches: int = 0
    fell_back: bool = False


def _check_fields(M, omega):
    if M.dim() != 3 or M.shape[0] != 3:
        raise ValueError("M must have shape (3, ny, nx)")
    if omega.shape != (2,) + tuple(M.shape[1:]):
        raise ValueError("omega must have shape (2, ny, nx)")
    if M.dtype != omega.dtype:
        raise TypeError("M and omega must share a dtype")
    if not (M.is_cuda and omega.is_cuda):
        raise ValueError("fields must be on the GPU")
    if not (M.is_contiguous() and omega.is_contiguous()):
        raise ValueError("fields must be contiguous")


def make_grid(nx, ny, h, src_idx, src_t=None) -> L.EikGrid:
    if src_idx.dtype != torch.int32 or not src_idx.is_cuda or not src_idx.is_contiguous():
        raise ValueError("src_idx must be a contiguous int32 GPU tensor")
    return L.EikGrid(int(nx), int(ny), float(h), int(src_idx.numel()), src_idx.data_ptr(),
                     None if src_t is None else src_t.data_ptr())


def workspace(grid: L.EikGrid, dtype_code: int, device) -> torch.Tensor:
    nbytes = L.lib().eik_workspace_bytes(ctypes.byref(grid), dtype_code)
    if nbytes == 0:
        L.check("eik_workspace_bytes", L.EIK_EINVAL)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


ADJ_RELAX, ADJ_LEVELS = 1, 2
LEVELS_CARRIED, LEVELS_AFTER = 1, 2


def tuning(tile_height=0, max_local_cycles=0, rounds_per_check=0, fast_cold_start=-1, adjoint_rounds=0,
           level_rounds=0, scheduler=0, node_lanes=0, adjoint_cycles=0, adjoint_waves=0, full_waves=0,
           adjoint_mode=0, level_mode=0):
    """Scheduling knobs (0 / -1 keep the library default). scheduler: 1 rounds,
    2 device work queue; node_lanes: 1, 2 or 4 lanes per node update;
    fast_cold_start: 0, 1 or 2 (four directions at once); adjoint_waves and
    full_waves: 1 or 4 (four directions at once); adjoint_mode: ADJ_RELAX
    (tile relaxation) or ADJ_LEVELS (level-ordered gather, needs levels);
    level_mode: LEVELS_CARRIED (the sweeps carry the levels) or LEVELS_AFTER
    (level rounds after sweeps that run as without levels)."""
    return L.EikTuning(tile_height, max_local_cycles, rounds_per_check, fast_cold_start, adjoint_rounds,
                       level_rounds, scheduler, node_lanes, adjoint_cycles, adjoint_waves, full_waves,
                       adjoint_mode, level_mode)


def solve(M, omega, src_idx, h, src_t=None, T_init=None, tol=1e-5, max_rounds=4096, check_feasible=False,
          tune=None, ws=None, time_kernels=False, levels=True, warm_fallback=False):
    """Forward solve. Returns (T, parent, level, Stats); level is None when
    ``levels`` is False (the adjoint does not need it). ``warm_fallback``
    (with T_init) drops a warm start that does not settle in two rounds and
    solves from the cold start instead (Stats.fell_back)."""
    _check_fields(M, omega)
    ny, nx = M.shape[1:]
    dev = M.device
    if src_t is not None:
        src_t = src_t.to(device=dev, dtype=M.dtype).contiguous()
    grid = make_grid(nx, ny, h, src_idx, src_t)
    dc = L.dtype_code(M)
    if ws is None:
        ws = workspace(grid, dc, dev)
    if tune is None:
        tune = autotune.lookup(nx * ny, autotune.dtype_name(M.dtype))
    T = torch.empty((ny, nx), dtype=M.dtype, device=dev)
    parent = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
    level = torch.empty((ny, nx), dtype=torch.int32, device=dev) if levels else None
    if T_init is not None:
        T_init = T_init.to(device=dev, dtype=M.dtype).contiguous()
    st = L.EikStats()
    rc = L.lib().eik_forward(ctypes.byref(grid), dc, L.ptr(M), L.ptr(omega), L.ptr(T_init), float(tol),
                             int(max_rounds),
                             (L.EIK_CHECK_FEASIBLE if check_feasible else 0) | (L.EIK_TIME_KERNELS if time_kernels else 0)
                             | (L.EIK_WARM_FALLBACK if warm_fallback else 0),
                             L.ptr(T),
                             L.ptr(parent), L.ptr(level), L.ptr(ws), ws.numel(),
                             None if tune is None else ctypes.byref(tune), ctypes.byref(st), L.stream_handle(dev))
    L.check("eik_forward", rc, ok=(L.EIK_OK, L.EIK_NOT_CONVERGED))
    return T, parent, level, stats_of(st)


def stats_of(st):
    """Stats from an eik_stats filled by a forward call."""
    return Stats(st.rounds, bool(st.converged), st.cell_updates, st.n_levels, st.status, st.sweep_launches,
                 st.sweep_ms, st.aux_rounds, st.fast_ms, st.fast_cell_updates, st.fast_launches, bool(st.fell_back))


def mixed_workspace(grid: L.EikGrid, device) -> torch.Tensor:
    nbytes = L.lib().eik_mixed_workspace_bytes(ctypes.byref(grid))
    if nbytes == 0:
        L.check("eik_mixed_workspace_bytes", L.EIK_EINVAL)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def solve_mixed(M, omega, src_idx, h, src_t=None, tol=1e-5, tol32=None, max_rounds=4096, check_feasible=False,
                tune32=None, tune=None, ws=None, time_kernels=False, levels=True):
    """Mixed-precision forward (eik_forward_mixed): FP32 sweeps from the cold
    start to ``tol32`` (default ``tol``) on FP32-rounded copies of the FP64
    fields, then FP64 sweeps from that field to ``tol``. Returns (T, parent,
    level, (Stats of the FP32 phase, Stats of the FP64 phase)) with T FP64."""
    _check_fields(M, omega)
    if M.dtype != torch.float64:
        raise TypeError("the mixed-precision solve takes FP64 fields")
    ny, nx = M.shape[1:]
    dev = M.device
    if src_t is not None:
        src_t = src_t.to(device=dev, dtype=torch.float64).contiguous()
    grid = make_grid(nx, ny, h, src_idx, src_t)
    if ws is None:
        ws = mixed_workspace(grid, dev)
    if tune32 is None:
        tune32 = autotune.lookup(nx * ny, "f32")
    T = torch.empty((ny, nx), dtype=torch.float64, device=dev)
    parent = torch.empty((ny, nx), dtype=torch.uint8, device=dev)
    level = torch.empty((ny, nx), dtype=torch.int32, device=dev) if levels else None
    st = (L.EikStats * 2)()
    rc = L.lib().eik_forward_mixed(ctypes.byref(grid), L.ptr(M), L.ptr(omega), float(tol if tol32 is None else tol32),
                                   float(tol), int(max_rounds),
                                   (L.EIK_CHECK_FEASIBLE if check_feasible else 0) |
                                   (L.EIK_TIME_KERNELS if time_kernels else 0),
                                   L.ptr(T), L.ptr(parent), L.ptr(level), L.ptr(ws), ws.numel(),
                                   None if tune32 is None else ctypes.byref(tune32),
                                   None if tune is None else ctypes.byref(tune), st, L.stream_handle(dev))
    L.check("eik_forward_mixed", rc, ok=(L.EIK_OK, L.EIK_NOT_CONVERGED))
    return T, parent, level, (stats_of(st[0]), stats_of(st[1]))


def adjoint(M, omega, T, parent, level, src_idx, h, dLdT, src_t=None, tune=None, ws=None, stats_out=None):
    """Backward pass. Returns (dL/dM, dL/domega, dL/dt_src); ``stats_out`` (a
    list) receives the call's Stats. ``level`` is not needed (may be None)."""
    _check_fields(M, omega)
    ny, nx = M.shape[1:]
    dev = M.device
    grid = make_grid(nx, ny, h, src_idx, src_t)
    dc = L.dtype_code(M)
    if ws is None:
        ws = workspace(grid, dc, dev)
    if tune is None:
        tune = autotune.lookup(nx * ny, autotune.dtype_name(M.dtype))
    dLdT = dLdT.to(dtype=M.dtype).contiguous()
    dM = torch.empty_like(M)
    dom = torch.empty_like(omega)
    ds = torch.empty(src_idx.numel(), dtype=M.dtype, device=dev)
    st = L.EikStats()
    rc = L.lib().eik_backward(ctypes.byref(grid), dc, L.ptr(M), L.ptr(omega), L.ptr(T), L.ptr(parent),
                              L.ptr(level), L.ptr(dLdT), L.ptr(dM), L.ptr(dom), L.ptr(ds), L.ptr(ws), ws.numel(),
                              None if tune is None else ctypes.byref(tune), ctypes.byref(st), L.stream_handle(dev))
    L.check("eik_backward", rc)
    if stats_out is not None:
        stats_out.append(Stats(st.rounds, bool(st.converged), 0, 0, rc, 0, 0.0, st.aux_rounds))
    return dM, dom, ds


def adjoint_mixed(M, omega, T, parent, src_idx, h, dLdT, src_t=None, tune=None, ws=None, stats_out=None,
                  level=None):
    """Backward pass of the mixed-precision state (eik_backward_mixed): FP64
    weights and parameter derivatives, FP32 adjoint relaxation (or the
    level-ordered gather with ``tune.adjoint_mode = ADJ_LEVELS`` and the
    forward's ``level``). Returns FP64 (dL/dM, dL/domega, dL/dt_src)."""
    _check_fields(M, omega)
    if M.dtype != torch.float64 or T.dtype != torch.float64:
        raise TypeError("the mixed-precision adjoint takes the FP64 fields and field T")
    ny, nx = M.shape[1:]
    dev = M.device
    grid = make_grid(nx, ny, h, src_idx, src_t)
    if ws is None:
        ws = mixed_workspace(grid, dev)
    if tune is None:
        tune = autotune.lookup(nx * ny, "f32")
    dLdT = dLdT.to(dtype=torch.float64).contiguous()
    dM = torch.empty_like(M)
    dom = torch.empty_like(omega)
    ds = torch.empty(src_idx.numel(), dtype=torch.float64, device=dev)
    st = L.EikStats()
    rc = L.lib().eik_backward_mixed(ctypes.byref(grid), L.ptr(M), L.ptr(omega), L.ptr(T), L.ptr(parent),
                                    L.ptr(level), L.ptr(dLdT), L.ptr(dM), L.ptr(dom), L.ptr(ds), L.ptr(ws), ws.numel(),
                                    None if tune is None else ctypes.byref(tune), ctypes.byref(st),
                                    L.stream_handle(dev))
    L.check("eik_backward_mixed", rc)
    if stats_out is not None:
        stats_out.append(Stats(st.rounds, bool(st.converged), 0, 0, rc, 0, 0.0, st.aux_rounds))
    return dM, dom, ds


class EikonalFn(torch.autograd.Function):
    """T = eikonal(M, omega, src_t); gradients by implicit differentiation."""

    @staticmethod
    def forward(ctx, M, omega, src_t, src_idx, h, tol, max_rounds, stats_sink=None, time_kernels=False,
                levels=False, mixed=False, tol32=None):
        M = M.contiguous()
        omega = omega.contiguous()
        if mixed:
            T, parent, level, st = solve_mixed(M, omega, src_idx, h, src_t=src_t, tol=tol, tol32=tol32,
                                               max_rounds=max_rounds, time_kernels=time_kernels, levels=levels)
            stats = st[1]
            if stats_sink is not None:
                stats_sink.extend(st)
        else:
            T, parent, level, stats = solve(M, omega, src_idx, h, src_t=src_t, tol=tol, max_rounds=max_rounds,
                                            time_kernels=time_kernels, levels=levels)
            if stats_sink is not None:
                stats_sink.append(stats)
        ctx.save_for_backward(M, omega, T, parent, src_idx)
        ctx.h = h
        ctx.mixed = mixed
        ctx.has_src_t = src_t is not None
        ctx.stats = stats
        ctx.mark_non_differentiable(parent)
        if level is not None:
            ctx.mark_non_differentiable(level)
        return T, parent, level

    @staticmethod
    def backward(ctx, gT, _gp=None, _gl=None):
        M, omega, T, parent, src_idx = ctx.saved_tensors
        if ctx.mixed:
            dM, dom, ds = adjoint_mixed(M, omega, T, parent, src_idx, ctx.h, gT)
        else:
            dM, dom, ds = adjoint(M, omega, T, parent, None, src_idx, ctx.h, gT)
        return dM, dom, (ds if ctx.has_src_t else None), None, None, None, None, None, None, None, None, None


# Tolerance of the FP64 phase of the mixed-precision solve when the caller
# asks for a looser one. The adjoint's donor weights are difference quotients
# of T at the grid scale, so the FP32 rounding the FP32 sweeps leave along the
# characteristics must be propagated out, not only recomputed locally: on the
# 2048^2 stress workload an FP64 phase stopped at 1e-5 leaves the gradient
# 8.0e-5 from the exact one (1.2e-4 in one run), at 3e-7 4.2e-5, at 1e-7
# 4.5e-6; the forward error falls from 6.7e-6 to 5.2e-7 at 3e-7.
MIXED_FP64_TOL = 3e-7


def eikonal(M, omega, src_idx, h, src_t=None, tol=1e-5, max_rounds=4096, stats_sink=None, time_kernels=False,
            levels=False, precision=None, tol32=None, tol64=None):
    """Differentiable solve; returns (T, parent, level) with level None unless
    ``levels`` is set. ``stats_sink`` (a list) receives the forward's Stats.

    precision None solves and differentiates in the dtype of M; "mixed" runs
    the mixed-precision forward (FP32 sweeps to ``tol32``, default ``tol``,
    then FP64 sweeps to ``tol64``, default min(tol, MIXED_FP64_TOL)) and the
    mixed adjoint (FP64 weights, FP32 relaxation): M, omega and src_t enter
    in FP64 (their gradients return in their own dtype), T is FP64, and
    ``stats_sink`` receives the Stats of both phases."""
    if precision not in (None, "mixed"):
        raise ValueError(f"precision {precision!r}: None or 'mixed'")
    mixed = precision == "mixed"
    if mixed:
        M, omega = M.to(torch.float64), omega.to(torch.float64)
        if src_t is not None:
            src_t = src_t.to(torch.float64)
        tol32 = tol if tol32 is None else tol32
        tol = min(tol, MIXED_FP64_TOL) if tol64 is None else tol64
    return EikonalFn.apply(M, omega, src_t, src_idx, h, tol, max_rounds, stats_sink, time_kernels, levels, mixed,
                           tol32)


def soft_workspace(grid: L.EikGrid, dtype_code: int, device) -> torch.Tensor:
    nbytes = L.lib().eik_soft_workspace_bytes(ctypes.byref(grid), dtype_code)
    if nbytes == 0:
        L.check("eik_soft_workspace_bytes", L.EIK_EINVAL)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def soft_solve(M, omega, src_idx, h, tau, src_t=None, tol=None, max_cycles=4096, ws=None):
    """Soft-min forward (eik_soft_forward): every stencil's segment minimum
    enters T = -tau log sum exp(-H_k / tau). Returns (T, cycles, converged).
    tol defaults to 1e-13 in FP64 and 1e-6 in FP32."""
    _check_fields(M, omega)
    ny, nx = M.shape[1:]
    dev = M.device
    if src_t is not None:
        src_t = src_t.to(device=dev, dtype=M.dtype).contiguous()
    grid = make_grid(nx, ny, h, src_idx, src_t)
    dc = L.dtype_code(M)
    if ws is None:
        ws = soft_workspace(grid, dc, dev)
    if tol is None:
        tol = 1e-13 if M.dtype == torch.float64 else 1e-6
    T = torch.empty((ny, nx), dtype=M.dtype, device=dev)
    cyc = ctypes.c_int32(0)
    rc = L.lib().eik_soft_forward(ctypes.byref(grid), dc, L.ptr(M), L.ptr(omega), float(tau), float(tol),
                                  int(max_cycles), L.ptr(T), L.ptr(ws), ws.numel(), ctypes.byref(cyc),
                                  L.stream_handle(dev))
    L.check("eik_soft_forward", rc, ok=(L.EIK_OK, L.EIK_NOT_CONVERGED))
    return T, cyc.value, rc == L.EIK_OK


def soft_adjoint(M, omega, T, src_idx, h, tau, dLdT, tol=None, max_cycles=4096, ws=None, cycles_out=None):
    """VJP of soft_solve's converged field (eik_soft_backward). Returns
    (dL/dM, dL/domega, dL/dt_src); ``cycles_out`` (a list) receives the
    relaxation cycles."""
    _check_fields(M, omega)
    ny, nx = M.shape[1:]
    dev = M.device
    grid = make_grid(nx, ny, h, src_idx)
    dc = L.dtype_code(M)
    if ws is None:
        ws = soft_workspace(grid, dc, dev)
    if tol is None:
        tol = 1e-13 if M.dtype == torch.float64 else 1e-6
    dLdT = dLdT.to(dtype=M.dtype).contiguous()
    T = T.contiguous()
    dM = torch.empty_like(M)
    dom = torch.empty_like(omega)
    ds = torch.empty(src_idx.numel(), dtype=M.dtype, device=dev)
    cyc = ctypes.c_int32(0)
    rc = L.lib().eik_soft_backward(ctypes.byref(grid), dc, L.ptr(M), L.ptr(omega), L.ptr(T), float(tau),
                                   L.ptr(dLdT), float(tol), int(max_cycles), L.ptr(dM), L.ptr(dom), L.ptr(ds),
                                   L.ptr(ws), ws.numel(), ctypes.byref(cyc), L.stream_handle(dev))
    L.check("eik_soft_backward", rc)
    if cycles_out is not None:
        cycles_out.append(cyc.value)
    return dM, dom, ds


class SoftEikonalFn(torch.autograd.Function):
    """T = soft-min eikonal(M, omega, src_t); the VJP solves the adjoint of the
    smooth fixed point."""

    @staticmethod
    def forward(ctx, M, omega, src_t, src_idx, h, tau, tol, max_cycles):
        M, omega = M.contiguous(), omega.contiguous()
        T, _, conv = soft_solve(M, omega, src_idx, h, tau, src_t=src_t, tol=tol, max_cycles=max_cycles)
        if not conv:
            raise RuntimeError("soft-min solve did not settle within max_cycles")
        ctx.save_for_backward(M, omega, T, src_idx)
        ctx.h, ctx.tau, ctx.tol, ctx.max_cycles = h, tau, tol, max_cycles
        ctx.has_src_t = src_t is not None
        return T

    @staticmethod
    def backward(ctx, gT):
        M, omega, T, src_idx = ctx.saved_tensors
        dM, dom, ds = soft_adjoint(M, omega, T, src_idx, ctx.h, ctx.tau, gT, tol=ctx.tol, max_cycles=ctx.max_cycles)
        return dM, dom, (ds if ctx.has_src_t else None), None, None, None, None, None


def soft_eikonal(M, omega, src_idx, h, tau, src_t=None, tol=None, max_cycles=4096):
    """Differentiable soft-min solve (Sec. 3.3's smooth stencil selection)."""
    return SoftEikonalFn.apply(M, omega, src_t, src_idx, h, tau, tol, max_cycles)


def _proj_params(eig_min, eig_max, eucl_clip, rho_max):
    return L.EikProjectParams(eig_min, eig_max, eucl_clip, rho_max)


def project(M, omega, eig_min=1e-3, eig_max=1e3, eucl_clip=1e3, rho_max=0.95):
    _check_fields(M, omega)
    n = M[0].numel()
    Mo, oo = torch.empty_like(M), torch.empty_like(omega)
    p = _proj_params(eig_min, eig_max, eucl_clip, rho_max)
    L.check("eik_project", L.lib().eik_project(n, L.dtype_code(M), L.ptr(M), L.ptr(omega), L.ptr(Mo), L.ptr(oo),
                                               ctypes.byref(p), L.stream_handle(M.device)))
    return Mo, oo


def project_backward(M, omega, gMo, goo, eig_min=1e-3, eig_max=1e3, eucl_clip=1e3, rho_max=0.95):
    _check_fields(M, omega)
    n = M[0].numel()
    gMo, goo = gMo.to(M.dtype).contiguous(), goo.to(M.dtype).contiguous()
    gM, go = torch.empty_like(M), torch.empty_like(omega)
    p = _proj_params(eig_min, eig_max, eucl_clip, rho_max)
    L.check("eik_project_backward",
            L.lib().eik_project_backward(n, L.dtype_code(M), L.ptr(M), L.ptr(omega), L.ptr(gMo), L.ptr(goo),
                                         L.ptr(gM), L.ptr(go), ctypes.byref(p), L.stream_handle(M.device)))
    return gM, go


class ProjectFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, M, omega, eig_min=1e-3, eig_max=1e3, eucl_clip=1e3, rho_max=0.95):
        M, omega = M.contiguous(), omega.contiguous()
        ctx.save_for_backward(M, omega)
        ctx.p = (eig_min, eig_max, eucl_clip, rho_max)
        return project(M, omega, *ctx.p)

    @staticmethod
    def backward(ctx, gMo, goo):
        M, omega = ctx.saved_tensors
        if gMo is None:
            gMo = torch.zeros_like(M)
        if goo is None:
            goo = torch.zeros_like(omega)
        gM, go = project_backward(M, omega, gMo, goo, *ctx.p)
        return gM, go, None, None, None, None
