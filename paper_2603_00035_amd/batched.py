"""Batched solving of many independent grids of different sizes.

The grids are packed one after the other (see include/eik.h): node arrays of
grid g start at node offset off_g, its metric planes at 3 off_g, its drift
planes at 2 off_g; source arrays hold the sources of grid 0, then grid 1, ...
with indices local to their grid.

``Batch`` plans the launch once (grid descriptors copied to the device), then
``forward`` / ``backward`` only enqueue kernels. With ``sync=False`` they run a
fixed round schedule with no host synchronisation, which makes the pair
capturable in a HIP graph (``torch.cuda.CUDAGraph``) and replayable;
``pending()`` then tells whether every phase settled within its budget.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from . import autotune
from .eikonal import MIXED_FP64_TOL, stats_of


class _Packed:
    """Shapes of a batch and the packing of its arrays (include/eik.h)."""

    def __init__(self, shapes, dtype, device):
        self.shapes = [(int(a), int(b), float(c), int(d)) for a, b, c, d in shapes]
        self.n_grids = len(self.shapes)
        self.dtype = dtype
        self.device = torch.device(device)
        G = L.EikGrid * self.n_grids
        self.grids = G(*[L.EikGrid(nx, ny, h, ns, None, None) for nx, ny, h, ns in self.shapes])
        sizes = [nx * ny for nx, ny, _, _ in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n_nodes = int(self.offsets[-1])
        self.src_offsets = np.concatenate([[0], np.cumsum([s[3] for s in self.shapes])]).astype(np.int64)
        self.n_src = int(self.src_offsets[-1])

    # -- packing helpers --------------------------------------------------
    def pack(self, Ms, oms):
        """Lists of (3, ny, nx) / (2, ny, nx) tensors -> packed flat tensors
        (each grid's block stays plane-major: [3][ny][nx], then the next grid)."""
        Mp = torch.cat([m.reshape(-1).to(self.device, self.dtype) for m in Ms])
        op = torch.cat([o.reshape(-1).to(self.device, self.dtype) for o in oms])
        return Mp.contiguous(), op.contiguous()

    def unpack_nodes(self, x):
        return [x[self.offsets[g]:self.offsets[g + 1]].reshape(self.shapes[g][1], self.shapes[g][0])
                for g in range(self.n_grids)]

    def unpack_planes(self, x, k):
        return [x[k * self.offsets[g]:k * self.offsets[g + 1]].reshape(k, self.shapes[g][1], self.shapes[g][0])
                for g in range(self.n_grids)]


class Batch(_Packed):
    def __init__(self, shapes, dtype=torch.float32, device="cuda", tune=None, max_rounds=64, mixed=False):
        """shapes: list of (nx, ny, h, n_src). ``mixed``: the mixed-precision
        calls (FP64 fields; FP32 sweeps with ``tune`` (default: the FP32 batch
        entry of the tuning table), then FP64 sweeps and the mixed adjoint
        with the library defaults at the same tile height)."""
        super().__init__(shapes, torch.float64 if mixed else dtype, device)
        self.mixed = bool(mixed)
        self.dc = L.EIK_MIXED if self.mixed else L.dtype_code(torch.empty(0, dtype=dtype))
        if tune is None:
            tune = autotune.lookup(sum(nx * ny for nx, ny, _, _ in self.shapes),
                                   "f32" if self.mixed else autotune.dtype_name(dtype), kind="batch")
        self.tune = tune
        self.tune64 = None
        if self.mixed:
            self.tune64 = L.EikTuning()
            self.tune64.tile_height = tune.tile_height if tune is not None else 0
        self.max_rounds = max_rounds
        nbytes = L.lib().eik_batch_workspace_bytes(self.n_grids, self.grids, self.dc)
        if nbytes == 0:
            L.check("eik_batch_workspace_bytes", L.EIK_EINVAL)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._tp = None if tune is None else ctypes.byref(tune)
        L.check("eik_batch_plan", L.lib().eik_batch_plan(self.n_grids, self.grids, self.dc, self._tp,
                                                           L.ptr(self.ws), self.ws.numel(),
                                                           L.stream_handle(self.device)))

    # -- calls ------------------------------------------------------------
    def alloc_forward(self, levels=False):
        T = torch.empty(self.n_nodes, dtype=self.dtype, device=self.device)
        parent = torch.empty(self.n_nodes, dtype=torch.uint8, device=self.device)
        level = torch.empty(self.n_nodes, dtype=torch.int32, device=self.device) if levels else None
        return T, parent, level

    def forward(self, M, om, src_idx, src_t=None, T_init=None, tol=1e-5, out=None, sync=True,
                time_kernels=False, levels=False, warm_fallback=False, tol32=None, tol64=None):
        """Returns (T, parent, level, Stats); level is None unless ``levels``
        (or an ``out`` triple with a level tensor) asks for it.
        ``warm_fallback`` (with T_init and sync) drops a warm start that does
        not settle in two rounds and solves from the cold start."""
        T, parent, level = out if out is not None else self.alloc_forward(levels)
        flags = L.EIK_TIME_KERNELS if (time_kernels and sync) else 0
        if self.mixed:
            if T_init is not None:
                raise ValueError("the mixed-precision batch solves from the cold start")
            st2 = (L.EikStats * 2)() if sync else None
            rc = L.lib().eik_forward_batched_mixed(
                self.n_grids, self.grids, L.ptr(src_idx), L.ptr(src_t), L.ptr(M), L.ptr(om),
                float(tol if tol32 is None else tol32), float(min(tol, MIXED_FP64_TOL) if tol64 is None else tol64),
                int(self.max_rounds), flags, L.ptr(T), L.ptr(parent), L.ptr(level), L.ptr(self.ws), self.ws.numel(),
                self._tp, ctypes.byref(self.tune64), st2, L.stream_handle(self.device))
            L.check("eik_forward_batched_mixed", rc, ok=(L.EIK_OK, L.EIK_NOT_CONVERGED))
            stats = None
            if st2 is not None:
                stats = stats_of(st2[1])
                stats.fp32 = stats_of(st2[0])
            return T, parent, level, stats
        st = L.EikStats() if sync else None
        if warm_fallback and sync:
            flags |= L.EIK_WARM_FALLBACK
        rc = L.lib().eik_forward_batched(self.n_grids, self.grids, self.dc, L.ptr(src_idx), L.ptr(src_t),
                                         L.ptr(M), L.ptr(om), L.ptr(T_init), float(tol), int(self.max_rounds),
                                         flags, L.ptr(T), L.ptr(parent), L.ptr(level), L.ptr(self.ws),
                                         self.ws.numel(), self._tp, None if st is None else ctypes.byref(st),
                                         L.stream_handle(self.device))
        L.check("eik_forward_batched", rc, ok=(L.EIK_OK, L.EIK_NOT_CONVERGED))
        stats = None
        if st is not None:
            stats = stats_of(st)
        return T, parent, level, stats

    def alloc_backward(self):
        dM = torch.empty(3 * self.n_nodes, dtype=self.dtype, device=self.device)
        dom = torch.empty(2 * self.n_nodes, dtype=self.dtype, device=self.device)
        ds = torch.empty(self.n_src, dtype=self.dtype, device=self.device)
        return dM, dom, ds

    def backward(self, M, om, T, parent, level, src_idx, dLdT, out=None, sync=True):
        dM, dom, ds = out if out is not None else self.alloc_backward()
        st = L.EikStats() if sync else None
        if self.mixed:
            rc = L.lib().eik_backward_batched_mixed(
                self.n_grids, self.grids, L.ptr(src_idx), L.ptr(M), L.ptr(om), L.ptr(T), L.ptr(parent), L.ptr(level),
                L.ptr(dLdT), L.ptr(dM), L.ptr(dom), L.ptr(ds), L.ptr(self.ws), self.ws.numel(), ctypes.byref(self.tune64),
                None if st is None else ctypes.byref(st), L.stream_handle(self.device))
            L.check("eik_backward_batched_mixed", rc)
            return dM, dom, ds, (None if st is None else st.rounds)
        rc = L.lib().eik_backward_batched(self.n_grids, self.grids, self.dc, L.ptr(src_idx), L.ptr(M), L.ptr(om),
                                          L.ptr(T), L.ptr(parent), L.ptr(level), L.ptr(dLdT), L.ptr(dM),
                                          L.ptr(dom), L.ptr(ds), L.ptr(self.ws), self.ws.numel(), self._tp,
                                          None if st is None else ctypes.byref(st), L.stream_handle(self.device))
        L.check("eik_backward_batched", rc)
        return dM, dom, ds, (None if st is None else st.rounds)

    def pending(self):
        """Tiles still flagged when the fixed budgets ran out (sweep, level, adjoint)."""
        out = (ctypes.c_int64 * 3)()
        L.check("eik_batch_pending", L.lib().eik_batch_pending(self.n_grids, self.grids, self.dc, L.ptr(self.ws),
                                                                 self.ws.numel(), out,
                                                                 L.stream_handle(self.device)))
        return tuple(int(v) for v in out)


class SoftBatch(_Packed):
    """Batched soft-min solves (eik_soft_forward_batched / _backward_batched):
    one workgroup per grid, each grid stopping at its own first quiet cycle."""

    def __init__(self, shapes, dtype=torch.float64, device="cuda"):
        super().__init__(shapes, dtype, device)
        self.dc = L.dtype_code(torch.empty(0, dtype=dtype))
        nbytes = L.lib().eik_soft_batch_workspace_bytes(self.n_grids, self.grids, self.dc)
        if nbytes == 0:
            L.check("eik_soft_batch_workspace_bytes", L.EIK_EINVAL)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def _tol(self, tol):
        return (1e-13 if self.dtype == torch.float64 else 1e-6) if tol is None else float(tol)

    def forward(self, M, om, src_idx, tau, src_t=None, tol=None, max_cycles=4096, out=None):
        """Packed fields -> (T packed, per-grid cycles, converged);
        ``self.last_cycle_ms`` receives the GPU time of the cycle launches."""
        T = out if out is not None else torch.empty(self.n_nodes, dtype=self.dtype, device=self.device)
        if src_t is not None:
            src_t = src_t.to(self.device, self.dtype).contiguous()
        cyc = (ctypes.c_int32 * self.n_grids)()
        ms = ctypes.c_double(0.0)
        rc = L.lib().eik_soft_forward_batched(self.n_grids, self.grids, self.dc, L.ptr(src_idx), L.ptr(src_t),
                                              L.ptr(M), L.ptr(om), float(tau), self._tol(tol), int(max_cycles),
                                              L.ptr(T), L.ptr(self.ws), self.ws.numel(), cyc, ctypes.byref(ms),
                                              L.stream_handle(self.device))
        L.check("eik_soft_forward_batched", rc, ok=(L.EIK_OK, L.EIK_NOT_CONVERGED))
        self.last_cycle_ms = ms.value
        return T, np.array(cyc[:], dtype=np.int32), rc == L.EIK_OK

    def backward(self, M, om, T, src_idx, tau, dLdT, tol=None, max_cycles=4096, out=None):
        """-> (dL/dM, dL/domega, dL/dt_src packed, per-grid cycles);
        ``self.last_adj_cycle_ms`` receives the GPU time of the cycle launches."""
        if out is None:
            out = (torch.empty_like(M), torch.empty_like(om),
                   torch.empty(self.n_src, dtype=self.dtype, device=self.device))
        dM, dom, ds = out
        dLdT = dLdT.to(self.dtype).contiguous()
        cyc = (ctypes.c_int32 * self.n_grids)()
        ms = ctypes.c_double(0.0)
        rc = L.lib().eik_soft_backward_batched(self.n_grids, self.grids, self.dc, L.ptr(src_idx), L.ptr(M),
                                               L.ptr(om), L.ptr(T), float(tau), L.ptr(dLdT), self._tol(tol),
                                               int(max_cycles), L.ptr(dM), L.ptr(dom), L.ptr(ds), L.ptr(self.ws),
                                               self.ws.numel(), cyc, ctypes.byref(ms), L.stream_handle(self.device))
        L.check("eik_soft_backward_batched", rc)
        self.last_adj_cycle_ms = ms.value
        return dM, dom, ds, np.array(cyc[:], dtype=np.int32)
