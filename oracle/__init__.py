"""Oracle: plain, slow, single-threaded FP64 CPU reference of the method.

TEST INFRASTRUCTURE. Only ``tests/``, the smoke check and the benchmark's CPU
baseline may import this package. It shares no code with the HIP library and
never imports it. The solve and the adjoint live in ``eik_oracle.c`` (plain C,
FP64, no fast-math, one thread); this module loads it with ctypes and adds two
brute-force references (Dijkstra on the 8-neighbour graph, the Hopf-Lax
minimisation of a two-point update) and the feasibility projection written
with plain PyTorch CPU float64 ops (its VJP is PyTorch autograd of that code).
"""
from __future__ import annotations

import ctypes
import heapq
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eik_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SOURCE = 0xFE
UNREACHED = 0xFF
NBX = (-1, -1, -1, 0, 1, 1, 1, 0)
NBY = (1, 0, -1, -1, -1, 0, 1, 1)


def build() -> str:
    """Compile the C oracle (always; a few seconds)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_ubyte)
        i, d = ctypes.c_int, ctypes.c_double
        L.ora_forward.argtypes = [i, i, d, dp, dp, i, ip, dp, dp, i, i, i, d, dp, ip]
        L.ora_forward.restype = i
        L.ora_local_update.argtypes = [i, i, d, dp, dp, dp, i, i, ip]
        L.ora_local_update.restype = d
        L.ora_two_point.argtypes = [dp, dp, d, i, i, d, d, dp, dp]
        L.ora_two_point.restype = i
        L.ora_one_point.argtypes = [dp, dp, d, i, d]
        L.ora_one_point.restype = d
        L.ora_local_update_all.argtypes = [i, i, d, dp, dp, dp, dp, up]
        L.ora_local_update_all.restype = None
        L.ora_candidate.argtypes = [i, i, d, dp, dp, dp, i, i, ip]
        L.ora_candidate.restype = d
        L.ora_parents_levels.argtypes = [i, i, d, dp, dp, i, ip, dp, up, ip]
        L.ora_vjp.argtypes = [i, i, d, dp, dp, i, ip, dp, up, dp, dp, dp, dp]
        L.ora_jvp.argtypes = [i, i, d, dp, dp, i, ip, dp, up, dp, dp, dp, dp]
        L.ora_soft_forward.argtypes = [i, i, d, dp, dp, i, ip, dp, d, i, d, dp, ip]
        L.ora_soft_forward.restype = i
        L.ora_soft_local.argtypes = [i, i, d, dp, dp, dp, d, i, dp, dp]
        L.ora_soft_local.restype = d
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _dp(a):
    return _p(a, ctypes.c_double)


def _ip(a):
    return _p(a, ctypes.c_int)


def forward(prob, mode="gs", one_point_only=False, tol=0.0, max_sweeps=100000, T_init=None):
    """Solve to stationarity (tol=0) or to the relative-change tolerance.

    mode "gs" (Gauss-Seidel four-ordering sweeps), "jacobi", or "gs_f32": the
    Gauss-Seidel sweeps with every stored value rounded to single precision
    (updates evaluated exactly in double), the best field a solve that stores
    T in single precision can reach; for measuring that storage's effect only.
    Returns (T[ny,nx], sweeps, status) with status 0 when converged."""
    modes = {"gs": 0, "jacobi": 1, "gs_f32": 2}
    M, om = _d(prob.M), _d(prob.omega)
    src = np.ascontiguousarray(prob.src_idx, np.int32)
    st = _d(prob.src_t)
    T = np.empty((prob.ny, prob.nx))
    sw = ctypes.c_int(0)
    Ti = None if T_init is None else _d(T_init)
    status = lib().ora_forward(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), src.size, _ip(src), _dp(st),
                               None if Ti is None else _dp(Ti), modes[mode],
                               int(one_point_only), int(max_sweeps), float(tol), _dp(T), ctypes.byref(sw))
    return T, sw.value, status


def parents_levels(prob, T):
    M, om, T = _d(prob.M), _d(prob.omega), _d(T)
    src = np.ascontiguousarray(prob.src_idx, np.int32)
    par = np.empty((prob.ny, prob.nx), np.uint8)
    lev = np.empty((prob.ny, prob.nx), np.int32)
    lib().ora_parents_levels(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), src.size, _ip(src), _dp(T),
                             _p(par, ctypes.c_ubyte), _ip(lev))
    return par, lev


def vjp(prob, T, parent, g):
    """dL/dM (3,ny,nx) w.r.t. stored scalars, dL/domega (2,ny,nx), dL/dt_src."""
    M, om, T, g = _d(prob.M), _d(prob.omega), _d(T), _d(g)
    src = np.ascontiguousarray(prob.src_idx, np.int32)
    par = np.ascontiguousarray(parent, np.uint8)
    dM = np.empty_like(M)
    dom = np.empty_like(om)
    ds = np.empty(src.size)
    lib().ora_vjp(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), src.size, _ip(src), _dp(T),
                  _p(par, ctypes.c_ubyte), _dp(g), _dp(dM), _dp(dom), _dp(ds))
    return dM, dom, ds


def jvp(prob, T, parent, dM, dom, dsrc=None):
    M, om, T = _d(prob.M), _d(prob.omega), _d(T)
    src = np.ascontiguousarray(prob.src_idx, np.int32)
    par = np.ascontiguousarray(parent, np.uint8)
    dT = np.empty((prob.ny, prob.nx))
    ds = _d(np.zeros(src.size) if dsrc is None else dsrc)
    lib().ora_jvp(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), src.size, _ip(src), _dp(T),
                  _p(par, ctypes.c_ubyte), _dp(_d(dM)), _dp(_d(dom)), _dp(ds), _dp(dT))
    return dT


def local_update(prob, T, c, one_point_only=False):
    M, om, T = _d(prob.M), _d(prob.omega), _d(T)
    code = ctypes.c_int(0)
    v = lib().ora_local_update(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), _dp(T), int(c),
                               int(one_point_only), ctypes.byref(code))
    return v, code.value


def local_update_all(prob, T):
    """The local update evaluated at every node of T (a Jacobi evaluation that
    changes nothing): (values [ny,nx], codes [ny,nx] uint8)."""
    M, om, T = _d(prob.M), _d(prob.omega), _d(T)
    v = np.empty((prob.ny, prob.nx))
    code = np.empty((prob.ny, prob.nx), np.uint8)
    lib().ora_local_update_all(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), _dp(T), _dp(v), _p(code, ctypes.c_ubyte))
    return v, code


def candidate(prob, T, c, code):
    """(value, valid) of one given candidate code at node c of the field T."""
    M, om, T = _d(prob.M), _d(prob.omega), _d(T)
    ok = ctypes.c_int(0)
    v = lib().ora_candidate(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), _dp(T), int(c), int(code),
                            ctypes.byref(ok))
    return v, bool(ok.value)


def two_point(g, b, h, kp, kq, Tp, Tq):
    g, b = _d(g), _d(b)
    t = ctypes.c_double(0)
    lam = np.zeros(2)
    ok = lib().ora_two_point(_dp(g), _dp(b), h, kp, kq, Tp, Tq, ctypes.byref(t), _dp(lam))
    return bool(ok), t.value, lam


def one_point(g, b, h, k, Tk):
    g, b = _d(g), _d(b)
    return lib().ora_one_point(_dp(g), _dp(b), h, k, Tk)


# --------------------------------------------------------------------------
# Brute-force references
# --------------------------------------------------------------------------

def dijkstra(prob):
    """Shortest arrival times on the directed 8-neighbour graph whose edge
    u -> v costs h (sqrt(m^T G_v m) + m . b_v) with m = x_v - x_u in grid units
    (the one-point update of Eq. one_point used as an edge weight)."""
    nx, ny, h = prob.nx, prob.ny, prob.h
    M, om = prob.M, prob.omega
    T = np.full(nx * ny, np.inf)
    pq = []
    for s, t in zip(prob.src_idx, prob.src_t):
        T[s] = t
        heapq.heappush(pq, (t, int(s)))
    done = np.zeros(nx * ny, bool)
    while pq:
        t, u = heapq.heappop(pq)
        if done[u]:
            continue
        done[u] = True
        ui, uj = u % nx, u // nx
        for k in range(8):
            vi, vj = ui - NBX[k], uj - NBY[k]  # u is neighbour k of v
            if not (0 <= vi < nx and 0 <= vj < ny):
                continue
            v = vj * nx + vi
            if done[v] or v in _src_set(prob):
                continue
            mx, my = -NBX[k] * h, -NBY[k] * h
            g11, g12, g22 = M[0, vj, vi], M[1, vj, vi], M[2, vj, vi]
            w = np.sqrt(g11 * mx * mx + 2 * g12 * mx * my + g22 * my * my) + mx * om[0, vj, vi] + my * om[1, vj, vi]
            if t + w < T[v]:
                T[v] = t + w
                heapq.heappush(pq, (T[v], v))
    return T.reshape(ny, nx)


_src_cache = {}


def _src_set(prob):
    key = id(prob)
    if key not in _src_cache:
        _src_cache.clear()
        _src_cache[key] = set(int(s) for s in prob.src_idx)
    return _src_cache[key]


def hopf_lax_two_point(g, b, h, kp, kq, Tp, Tq, n=200001):
    """Two-point update as the minimum over the segment between the donors of
    (1-t) T_p + t T_q + h F((1-t) m_p + t m_q), F(v) = |v|_G + b.v, found by a
    dense scan of t in [0, 1] (independent of the quadratic formula)."""
    t = np.linspace(0.0, 1.0, n)
    mpx, mpy = -NBX[kp], -NBY[kp]
    mqx, mqy = -NBX[kq], -NBY[kq]
    vx = (1 - t) * mpx + t * mqx
    vy = (1 - t) * mpy + t * mqy
    F = np.sqrt(g[0] * vx * vx + 2 * g[1] * vx * vy + g[2] * vy * vy) + b[0] * vx + b[1] * vy
    val = (1 - t) * Tp + t * Tq + h * F
    a = int(np.argmin(val))
    return val[a], t[a]


def closed_form(prob_const, sources_xy):
    """T(x) = min_s sqrt(d^T G d) + b^T d, d = x - s, for constant G, b
    (substitution into Eq. randers_eikonal)."""
    nx, ny, h = prob_const.nx, prob_const.ny, prob_const.h
    g11, g12, g22 = (prob_const.M[k, 0, 0] for k in range(3))
    bx, by = prob_const.omega[0, 0, 0], prob_const.omega[1, 0, 0]
    X, Y = np.meshgrid(np.arange(nx) * h, np.arange(ny) * h)
    best = np.full((ny, nx), np.inf)
    for (si, sj) in sources_xy:
        dx, dy = X - si * h, Y - sj * h
        best = np.minimum(best, np.sqrt(g11 * dx * dx + 2 * g12 * dx * dy + g22 * dy * dy) + bx * dx + by * dy)
    return best


# --------------------------------------------------------------------------
# Feasibility projection (App. learning details, "Feasibility Projections")
# --------------------------------------------------------------------------

def project_torch(M, om, eig_min=1e-3, eig_max=1e3, eucl_clip=1e3, rho_max=0.95):
    """Plain PyTorch float64 projection; M (3, ...), om (2, ...) tensors.

    Eigenvalues by the trace-discriminant formula, clamped to [eig_min,
    eig_max]; when a clamp is active G is rebuilt as U diag U^T with the
    principal angle atan2(2 g12, g11 - g22)/2, otherwise G passes unchanged.
    The drift is clipped to Euclidean norm eucl_clip and then rescaled to
    rho_max when |b|_{G^-1} exceeds rho_max."""
    import torch
    g11, g12, g22 = M[0], M[1], M[2]
    tr, dif = g11 + g22, g11 - g22
    disc = torch.sqrt(dif * dif + 4 * g12 * g12)
    lp, lm = 0.5 * (tr + disc), 0.5 * (tr - disc)
    lpc, lmc = lp.clamp(eig_min, eig_max), lm.clamp(eig_min, eig_max)
    clamped = (lpc != lp) | (lmc != lm)
    th = 0.5 * torch.atan2(2 * g12, dif)
    c, s = torch.cos(th), torch.sin(th)
    r11 = lpc * c * c + lmc * s * s
    r12 = (lpc - lmc) * c * s
    r22 = lpc * s * s + lmc * c * c
    n11 = torch.where(clamped, r11, g11)
    n12 = torch.where(clamped, r12, g12)
    n22 = torch.where(clamped, r22, g22)
    b1, b2 = om[0], om[1]
    e = torch.sqrt(b1 * b1 + b2 * b2)
    sc = torch.where(e > eucl_clip, eucl_clip / torch.where(e > 0, e, torch.ones_like(e)), torch.ones_like(e))
    b1, b2 = b1 * sc, b2 * sc
    det = n11 * n22 - n12 * n12
    rho = torch.sqrt((b1 * b1 * n22 - 2 * b1 * b2 * n12 + b2 * b2 * n11) / det)
    sr = torch.where(rho > rho_max, rho_max / torch.where(rho > 0, rho, torch.ones_like(rho)), torch.ones_like(rho))
    return torch.stack([n11, n12, n22]), torch.stack([b1 * sr, b2 * sr])


def project(M, om, **kw):
    import torch
    Mo, oo = project_torch(torch.from_numpy(_d(M)), torch.from_numpy(_d(om)), **kw)
    return Mo.numpy(), oo.numpy()


def project_vjp(M, om, gM, gom, **kw):
    import torch
    Mt = torch.from_numpy(_d(M)).requires_grad_(True)
    ot = torch.from_numpy(_d(om)).requires_grad_(True)
    Mo, oo = project_torch(Mt, ot, **kw)
    (Mo * torch.from_numpy(_d(gM))).sum().add((oo * torch.from_numpy(_d(gom))).sum()).backward()
    return Mt.grad.numpy(), ot.grad.numpy()


# -- soft-min mode -------------------------------------------------------------
# The smooth alternative to stencil selection the paper names (Sec. 3.3): each
# stencil contributes the minimum of the Hopf-Lax objective over its segment
# (its two-point value when both barycentric coordinates are >= 0, else the
# smaller one-point value of its endpoints), and a node takes the soft minimum
# -tau log sum exp(-H_k / tau) over its eight stencils.

def soft_forward(prob, tau, tol=1e-14, max_sweeps=100000):
    """Gauss-Seidel sweeps of the soft update from +inf until a full cycle
    changes no node by more than tol (relative). Returns (T, sweeps, status)."""
    M, om = _d(prob.M), _d(prob.omega)
    src = np.ascontiguousarray(prob.src_idx, np.int32)
    st = _d(prob.src_t)
    T = np.empty((prob.ny, prob.nx))
    sw = ctypes.c_int(0)
    status = lib().ora_soft_forward(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), src.size, _ip(src), _dp(st),
                                    float(tau), int(max_sweeps), float(tol), _dp(T), ctypes.byref(sw))
    return T, sw.value, status


def soft_local(prob, T, tau, c):
    """(value, coef[8], dth[5]) of the soft update at node c: its derivatives
    with respect to the eight neighbour times and the stored parameters."""
    M, om, T = _d(prob.M), _d(prob.omega), _d(T)
    coef = np.zeros(8)
    dth = np.zeros(5)
    v = lib().ora_soft_local(prob.nx, prob.ny, prob.h, _dp(M), _dp(om), _dp(T), float(tau), int(c), _dp(coef),
                             _dp(dth))
    return v, coef, dth


def soft_vjp(prob, T, tau, g):
    """Vector-Jacobian product of the soft fixed point T = F(T, theta): the
    adjoint lambda solves (I - J^T) lambda = g, J_ij = dF_i/dT_j (sources and
    unreached nodes have empty rows), with a sparse direct solve (scipy); then
    dL/dtheta_i = lambda_i dF_i/dtheta_i and dL/dt_s = lambda_s. Returns
    (dL/dM (3,ny,nx) w.r.t. the stored scalars, dL/domega (2,ny,nx), dL/dt_src)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    nx, ny = prob.nx, prob.ny
    n = nx * ny
    NBX = (-1, -1, -1, 0, 1, 1, 1, 0)
    NBY = (1, 0, -1, -1, -1, 0, 1, 1)
    T = _d(T)
    src = set(int(c) for c in np.asarray(prob.src_idx).ravel())
    reach = np.isfinite(T.ravel())
    rows, cols, vals = [], [], []
    dth = np.zeros((5, n))
    for c in range(n):
        if c in src or not reach[c]:
            continue
        _, coef, d5 = soft_local(prob, T, tau, c)
        dth[:, c] = d5
        i, j = c % nx, c // nx
        for k in range(8):
            if coef[k] != 0.0:
                rows.append(c)
                cols.append((j + NBY[k]) * nx + (i + NBX[k]))
                vals.append(coef[k])
    J = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A = (sp.identity(n, format="csr") - J.T).tocsc()
    gg = np.where(reach, _d(g).ravel(), 0.0)
    keep = np.nonzero(reach)[0]
    lam = np.zeros(n)
    lam[keep] = spla.spsolve(A[keep][:, keep], gg[keep])
    grad = lam * dth
    dM = grad[:3].reshape(3, ny, nx)
    dom = grad[3:].reshape(2, ny, nx)
    ds = np.array([lam[int(c)] for c in np.asarray(prob.src_idx).ravel()])
    return dM, dom, ds
