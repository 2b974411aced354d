"""GPU parity of the inverse-problem kernels (total variation, data term, sum
of squares, parameter step) against the oracle, and of whole recovery
iterations against the same iterations composed from the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import inverse_ref as I
from synthetic.fields import Problem
from tests.gpu_common import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def lib():
    from paper_2603_00035_amd import _lib as L
    return L, L.lib()


def scratch(dev):
    L, lb = lib()
    return torch.empty(lb.eik_inv_scratch_bytes(), dtype=torch.uint8, device=dev)


@pytest.mark.parametrize("dt,rtol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("C,ny,nx", [(1, 1, 70), (2, 65, 1), (3, 37, 53), (4, 480, 600), (3, 1, 1)])
def test_tv_matches_oracle(dt, rtol, C, ny, nx):
    L, lb = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(C * 1000 + nx)
    F = rng.normal(size=(C, ny, nx))
    F[:, : ny // 3, : nx // 3] = 0.25  # a flat block: zero norms take the subgradient 0
    w = rng.uniform(0.5, 2.0, C)
    g0 = rng.normal(size=F.shape)
    say(f"[tv] {C} planes {nx}x{ny} {dt}")
    Fd = torch.tensor(F, dtype=dt, device=dev)
    if dt == torch.float32:
        F = Fd.double().cpu().numpy()
    gd = torch.tensor(g0, dtype=dt, device=dev)
    val = torch.zeros(1, dtype=torch.float64, device=dev)
    wc = (ctypes.c_double * C)(*w)
    rc = lb.eik_tv(nx, ny, C, L.dtype_code(Fd), L.ptr(Fd), wc, 0.3, L.ptr(gd), val.data_ptr(),
                   L.ptr(scratch(dev)), L.stream_handle(dev))
    assert rc == 0
    vo, go = I.tv(F, w)
    torch.cuda.synchronize()
    assert float(val) == pytest.approx(0.3 * vo, rel=rtol, abs=1e-12)
    want = g0.astype(np.float64) + 0.3 * go
    if dt == torch.float32:
        want = torch.tensor(g0, dtype=dt).double().numpy() + 0.3 * go
    got = gd.double().cpu().numpy()
    assert np.max(np.abs(got - want)) <= rtol * (1 + np.max(np.abs(want))) * (1 if dt == torch.float64 else 10)


@pytest.mark.parametrize("dt,rtol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("ny,nx,iso", [(37, 53, 0.0), (64, 70, 0.3), (1, 90, 0.5), (480, 600, 0.1)])
def test_tv_log_euclid_matches_oracle(dt, rtol, ny, nx, iso):
    """Random SPD metrics, a share of them isotropic (coinciding eigenvalues,
    where the logarithm's divided difference takes its limit), and a block of
    constant metric (zero norms, subgradient 0)."""
    L, lb = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(nx + ny)
    A = rng.normal(size=(ny, nx, 2, 2))
    G = A @ np.swapaxes(A, -1, -2) + 0.3 * np.eye(2)
    sel = rng.uniform(size=(ny, nx)) < iso
    G[sel] = rng.uniform(0.5, 2.0, size=(ny, nx))[sel][:, None, None] * np.eye(2)
    G[: ny // 4, : nx // 4] = np.array([[1.3, 0.2], [0.2, 0.7]])
    M = np.stack([G[..., 0, 0], G[..., 0, 1], G[..., 1, 1]])
    say(f"[tv log-euclid] {nx}x{ny} {dt}, isotropic share {iso}")
    Md = torch.tensor(M, dtype=dt, device=dev)
    if dt == torch.float32:
        M = Md.double().cpu().numpy()
    g0 = rng.normal(size=M.shape)
    gd = torch.tensor(g0, dtype=dt, device=dev)
    val = torch.zeros(1, dtype=torch.float64, device=dev)
    work = torch.empty(lb.eik_tv_log_euclid_work_bytes(nx, ny, L.dtype_code(Md)), dtype=torch.uint8, device=dev)
    rc = lb.eik_tv_log_euclid(nx, ny, L.dtype_code(Md), L.ptr(Md), 0.3, L.ptr(gd), val.data_ptr(), L.ptr(work),
                              L.ptr(scratch(dev)), L.stream_handle(dev))
    assert rc == 0
    vo, go = I.tv_log_euclid(M)
    torch.cuda.synchronize()
    assert float(val) == pytest.approx(0.3 * vo, rel=rtol * (1 if dt == torch.float64 else 10))
    want = torch.tensor(g0, dtype=dt).double().numpy() + 0.3 * go
    got = gd.double().cpu().numpy()
    err = np.max(np.abs(got - want)) / (1 + np.max(np.abs(want)))
    say(f"  value {float(val):.6e} vs {0.3 * vo:.6e}, gradient max rel {err:.2e}")
    assert err <= rtol * (1 if dt == torch.float64 else 10)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_obs_loss_and_sum_sq_match_oracle(dt):
    L, lb = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    n = 300_001  # more than one pass of the fixed grid
    T = rng.uniform(0, 3, n)
    To = rng.uniform(0, 3, n)
    T[::97] = np.inf
    To[::101] = np.inf
    mask = (rng.uniform(size=n) < 0.3).astype(np.uint8)
    Td, Tod = torch.tensor(T, dtype=dt, device=dev), torch.tensor(To, dtype=dt, device=dev)
    md = torch.tensor(mask, device=dev)
    g = torch.empty_like(Td)
    val = torch.zeros(2, dtype=torch.float64, device=dev)
    sc = scratch(dev)
    st = L.stream_handle(dev)
    say(f"[obs loss] n={n} {dt}")
    assert lb.eik_obs_loss(n, L.dtype_code(Td), L.ptr(Td), L.ptr(Tod), L.ptr(md), L.ptr(g), val.data_ptr(),
                           L.ptr(sc), st) == 0
    assert lb.eik_sum_sq(n, L.dtype_code(g), L.ptr(g), val.data_ptr() + 8, L.ptr(sc), st) == 0
    assert lb.eik_sum_sq(n, L.dtype_code(g), L.ptr(g), val.data_ptr() + 8, L.ptr(sc), st) == 0  # accumulates
    torch.cuda.synchronize()
    vo, go = I.obs_loss(Td.double().cpu().numpy(), Tod.double().cpu().numpy(), mask)
    tol = 1e-12 if dt == torch.float64 else 1e-6
    assert float(val[0]) == pytest.approx(vo, rel=tol)
    assert np.allclose(g.double().cpu().numpy(), go, rtol=tol, atol=0)
    assert float(val[1]) == pytest.approx(2 * float(np.sum(g.double().cpu().numpy() ** 2)), rel=1e-12)


@pytest.mark.parametrize("method,max_norm", [(0, 0.0), (1, 0.0), (1, 0.5), (0, 0.5)])
def test_param_step_matches_oracle(method, max_norm):
    L, lb = lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(method * 10 + int(max_norm * 10))
    n = 5000
    p = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    pd_, md_, vd_ = (torch.tensor(x, device=dev) for x in (p, m, v))
    gsq = torch.zeros(1, dtype=torch.float64, device=dev)
    say(f"[param step] method={method} max_norm={max_norm}")
    for t in range(1, 5):
        g = rng.normal(size=n) * (0.1 if t % 2 else 3.0)
        gd = torch.tensor(g, device=dev)
        gsq.fill_(float(np.sum(g * g)))
        assert lb.eik_param_step(n, L.dtype_code(pd_), method, L.ptr(pd_), L.ptr(gd), L.ptr(md_), L.ptr(vd_), 0.01,
                                 0.9, 0.999, 1e-8, t, max_norm, gsq.data_ptr(), L.stream_handle(dev)) == 0
        p, m, v = I.param_step(method, p, g, m, v, 0.01, 0.9, 0.999, 1e-8, t, max_norm, float(np.sum(g * g)))
    torch.cuda.synchronize()
    assert np.allclose(pd_.cpu().numpy(), p, rtol=1e-13, atol=1e-15)


def _isotropic_case(nx, ny, obs_frac, seed):
    """The paper's isotropic recovery problem: G = g I with g = 1 on the left
    half and 2 on the right, one source at the centre, zero drift."""
    h = 1.0 / (nx - 1)
    g = np.where(np.arange(nx)[None, :] < nx // 2, 1.0, 2.0) * np.ones((ny, 1))
    M = np.stack([g, np.zeros_like(g), g])
    om = np.zeros((2, ny, nx))
    src = np.array([(ny // 2) * nx + nx // 2], np.int32)
    truth = Problem(nx, ny, h, M, om, src, np.zeros(1))
    T_obs, _, st = oracle.forward(truth)
    assert st == 0
    mask = (np.random.default_rng(seed).uniform(size=(ny, nx)) < obs_frac).astype(np.uint8)
    M0 = np.stack([np.full_like(g, 1.5), np.zeros_like(g), np.full_like(g, 1.5)])
    return truth, T_obs, mask, M0, om


def _oracle_iterations(truth, T_obs, mask, M0, om0, cfg, iters):
    from paper_2603_00035_amd import inverse as V
    M, om = M0.copy(), om0.copy()
    mM, vM, mo, vo = (np.zeros_like(M), np.zeros_like(M), np.zeros_like(om), np.zeros_like(om))
    for k in range(iters):
        prob = Problem(truth.nx, truth.ny, truth.h, M, om, truth.src_idx, truth.src_t)
        T, _, _ = oracle.forward(prob, tol=cfg.tol)
        par, _ = oracle.parents_levels(prob, T)
        _, g = I.obs_loss(T, T_obs, mask)
        gM, gom, _ = oracle.vjp(prob, T, par, g)
        if cfg.tv_metric == "log_euclid":
            gM = gM + cfg.lam_G * I.tv_log_euclid(M)[1]
        else:
            gM = gM + cfg.lam_G * I.tv(M, V.G_WEIGHTS)[1]
        gom = gom + cfg.lam_b * I.tv(om, V.B_WEIGHTS)[1]
        gsq = float(np.sum(gM * gM) + np.sum(gom * gom))
        method = 1 if cfg.method == "adam" else 0
        M, mM, vM = I.param_step(method, M, gM, mM, vM, V.lr_at(cfg, cfg.lr_G, k, iters), cfg.beta1, cfg.beta2,
                                 cfg.eps, k + 1, cfg.max_norm, gsq)
        om, mo, vo = I.param_step(method, om, gom, mo, vo, V.lr_at(cfg, cfg.lr_b, k, iters), cfg.beta1, cfg.beta2,
                                  cfg.eps, k + 1, cfg.max_norm, gsq)
        if cfg.isotropic:
            M = I.tie_isotropic(M)
        M, om = oracle.project(M, om, eig_min=cfg.eig_min, eig_max=cfg.eig_max, eucl_clip=cfg.eucl_clip,
                               rho_max=cfg.rho_max)
    return M, om


# Whole iterations are compared where their outcome is a smooth function of
# the arithmetic: the TV subgradient of a nearly flat field points wherever
# rounding puts it, and Adam turns any such direction into a full step, so TV
# enters only from a rough initial field (its kernel is checked exactly above).
@pytest.mark.parametrize("method,max_norm,lam_G,rough,iso,tvm", [("adam", 0.5, 0.0, False, False, "frobenius"),
                                                                  ("gd", 0.0, 0.0, False, False, "frobenius"),
                                                                  ("gd", 0.0, 1e-2, True, False, "frobenius"),
                                                                  ("adam", 0.0, 1e-2, True, False, "frobenius"),
                                                                  ("adam", 0.5, 0.0, False, True, "frobenius"),
                                                                  ("gd", 0.0, 1e-2, True, False, "log_euclid"),
                                                                  ("adam", 0.0, 1e-2, True, False, "log_euclid")])
def test_recovery_iterations_match_the_oracle(method, max_norm, lam_G, rough, iso, tvm):
    from paper_2603_00035_amd import inverse as V
    truth, T_obs, mask, M0, om0 = _isotropic_case(41, 37, 0.4, 1)
    if rough:
        M0 = M0 * np.random.default_rng(2).uniform(0.8, 1.2, M0.shape)
        M0[1] = 0.0
        if tvm == "log_euclid":  # a rotated, anisotropic start so that log G is not diagonal
            M0[1] = np.random.default_rng(3).uniform(-0.3, 0.3, M0[1].shape)
    cfg = V.InverseConfig(method=method, max_norm=max_norm, lam_G=lam_G, lam_b=0.0, lr_G=0.05, lr_b=0.02,
                          isotropic=iso, tv_metric=tvm)
    iters = 4
    say(f"[recovery] {method} clip={max_norm} lam_G={lam_G} rough={rough} 41x37, {iters} iterations vs the oracle")
    dev = torch.device("cuda:0")
    R = V.Recovery(torch.tensor(M0, device=dev), torch.tensor(om0, device=dev),
                   torch.tensor(truth.src_idx, device=dev), truth.h, torch.tensor(T_obs, device=dev),
                   torch.tensor(mask, device=dev), cfg)
    hist = R.run(iters)
    Mo, oo = _oracle_iterations(truth, T_obs, mask, M0, om0, cfg, iters)
    rel = max(np.max(np.abs(R.M.cpu().numpy() - Mo)) / np.max(np.abs(Mo)),
              np.max(np.abs(R.om.cpu().numpy() - oo)) / max(1e-30, np.max(np.abs(oo))))
    say(f"  max rel difference {rel:.2e}; data loss {float(hist[0, 0]):.3e} -> {float(hist[-1, 0]):.3e}")
    assert rel <= 1e-8
    assert float(hist[-1, 0]) < float(hist[0, 0])


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_isotropic_tie_matches_oracle(dt):
    L, lb = lib()
    dev = torch.device("cuda:0")
    M = np.random.default_rng(4).normal(size=(3, 33, 70))
    Md = torch.tensor(M, dtype=dt, device=dev)
    Mh = Md.double().cpu().numpy()
    assert lb.eik_tie_isotropic(33 * 70, L.dtype_code(Md), L.ptr(Md), L.stream_handle(dev)) == 0
    torch.cuda.synchronize()
    assert np.array_equal(Md.double().cpu().numpy(), I.tie_isotropic(Mh).astype(
        np.float32 if dt == torch.float32 else np.float64).astype(np.float64))


def test_isotropic_recovery_reaches_the_paper_accuracy():
    """Sec. 5, isotropic metric recovery: g = 1 | 2 on an 80 x 80 grid, one
    source, full observations, the paper's step size 1e-2 and TV weight 1e-3,
    300 iterations (Adam, cosine schedule); the paper reports 5.6 % relative
    error. Observations come from the oracle's solve of the true field."""
    from paper_2603_00035_amd import inverse as V
    truth, T_obs, mask, M0, om0 = _isotropic_case(80, 80, 1.0, 0)
    dev = torch.device("cuda:0")
    cfg = V.InverseConfig(lam_G=1e-3, lr_G=1e-2, free_drift=False, isotropic=True)
    R = V.Recovery(torch.tensor(M0, device=dev), torch.tensor(om0, device=dev),
                   torch.tensor(truth.src_idx, device=dev), truth.h, torch.tensor(T_obs, device=dev),
                   torch.tensor(mask, device=dev), cfg)
    hist = R.run(300)
    g = truth.M[0]
    err = float(np.linalg.norm(R.M[0].cpu().numpy() - g) / np.linalg.norm(g))
    say(f"[recovery] isotropic 80x80, 300 iterations: relative error {err:.4f} (paper 0.056), "
        f"data loss {float(hist[0, 0]):.3e} -> {float(hist[-1, 0]):.3e}")
    assert err <= 0.08


def _multi_case(nx, ny, obs_frac, seed, sites):
    """The isotropic problem observed from several fires, one ignition each."""
    truth, _, _, M0, om0 = _isotropic_case(nx, ny, obs_frac, seed)
    fires, T_obs, masks = [], [], []
    rng = np.random.default_rng(seed + 100)
    for (i, j) in sites:
        p = Problem(nx, ny, truth.h, truth.M, truth.omega, np.array([j * nx + i], np.int32), np.zeros(1))
        T, _, st = oracle.forward(p)
        assert st == 0
        fires.append(p)
        T_obs.append(T)
        masks.append((rng.uniform(size=(ny, nx)) < obs_frac).astype(np.uint8))
    return truth, fires, np.stack(T_obs), np.stack(masks), M0, om0


def _oracle_multi_iterations(fires, T_obs, masks, M0, om0, cfg, iters):
    from paper_2603_00035_amd import inverse as V
    M, om = M0.copy(), om0.copy()
    mM, vM, mo, vo = (np.zeros_like(M), np.zeros_like(M), np.zeros_like(om), np.zeros_like(om))
    f0 = fires[0]
    for k in range(iters):
        gM, gom = np.zeros_like(M), np.zeros_like(om)
        for f, To, mk in zip(fires, T_obs, masks):
            prob = Problem(f0.nx, f0.ny, f0.h, M, om, f.src_idx, f.src_t)
            T, _, _ = oracle.forward(prob, tol=cfg.tol)
            par, _ = oracle.parents_levels(prob, T)
            _, g = I.obs_loss(T, To, mk)
            a, b, _ = oracle.vjp(prob, T, par, g)
            gM, gom = gM + a, gom + b
        if cfg.tv_metric == "log_euclid":
            gM = gM + cfg.lam_G * I.tv_log_euclid(M)[1]
        else:
            gM = gM + cfg.lam_G * I.tv(M, V.G_WEIGHTS)[1]
        gom = gom + cfg.lam_b * I.tv(om, V.B_WEIGHTS)[1]
        gsq = float(np.sum(gM * gM) + np.sum(gom * gom))
        method = 1 if cfg.method == "adam" else 0
        M, mM, vM = I.param_step(method, M, gM, mM, vM, V.lr_at(cfg, cfg.lr_G, k, iters), cfg.beta1, cfg.beta2,
                                 cfg.eps, k + 1, cfg.max_norm, gsq)
        om, mo, vo = I.param_step(method, om, gom, mo, vo, V.lr_at(cfg, cfg.lr_b, k, iters), cfg.beta1, cfg.beta2,
                                  cfg.eps, k + 1, cfg.max_norm, gsq)
        if cfg.isotropic:
            M = I.tie_isotropic(M)
        M, om = oracle.project(M, om, eig_min=cfg.eig_min, eig_max=cfg.eig_max, eucl_clip=cfg.eucl_clip,
                               rho_max=cfg.rho_max)
    return M, om


@pytest.mark.parametrize("method,lam_G,rough,iso", [("gd", 0.0, False, False), ("adam", 1e-2, True, False),
                                                    ("adam", 0.0, False, True)])
def test_multi_source_iterations_match_the_oracle(method, lam_G, rough, iso):
    """Sec. 5, multi-source recovery: K fires with different ignitions solved
    and differentiated in one batched launch, gradients summed; whole
    iterations against the oracle's per-fire solves and VJPs."""
    from paper_2603_00035_amd import inverse as V
    sites = [(20, 18), (5, 6), (34, 30)]
    truth, fires, T_obs, masks, M0, om0 = _multi_case(41, 37, 0.4, 3, sites)
    if rough:
        M0 = M0 * np.random.default_rng(5).uniform(0.8, 1.2, M0.shape)
        M0[1] = 0.0
    cfg = V.InverseConfig(method=method, lam_G=lam_G, lam_b=0.0, lr_G=0.05, lr_b=0.02, isotropic=iso)
    iters = 3
    say(f"[recovery] {len(sites)} fires, {method} lam_G={lam_G} rough={rough} iso={iso}, {iters} iterations")
    dev = torch.device("cuda:0")
    srcs = [torch.tensor(f.src_idx, device=dev) for f in fires]
    R = V.MultiRecovery(torch.tensor(M0, device=dev), torch.tensor(om0, device=dev), srcs, truth.h,
                        torch.tensor(T_obs, device=dev), torch.tensor(masks, device=dev), cfg)
    hist = R.run(iters)
    Mo, oo = _oracle_multi_iterations(fires, T_obs, masks, M0, om0, cfg, iters)
    rel = max(np.max(np.abs(R.M.cpu().numpy() - Mo)) / np.max(np.abs(Mo)),
              np.max(np.abs(R.om.cpu().numpy() - oo)) / max(1e-30, np.max(np.abs(oo))))
    say(f"  max rel difference {rel:.2e}; data loss {float(hist[0, 0]):.3e} -> {float(hist[-1, 0]):.3e}")
    assert rel <= 1e-8
    assert float(hist[-1, 0]) < float(hist[0, 0])
