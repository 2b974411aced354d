"""The covariate encoder on the GPU against its oracle: the dense and
combination kernels element by element, the whole encoder forward, and the
hybrid gradient of one training step (network, projection, solve, data term,
implicit adjoint, projection VJP, encoder backward) against the oracle's
chain with an FP64 solve.

Tolerances from the arithmetic: FP32 sums of K terms are within
K 2^-24 sum|terms| of the exact sum; the encoder stores activations and their
gradients in bfloat16 (2^-9 relative), and an FP32 accumulation can round a
value to the neighbouring bfloat16 when it lies within K 2^-24 of a rounding
boundary (about 2 % of the values of a 576-term convolution), so whole-network
outputs and gradients are compared in relative L2 at the level such flips
reach (1e-2), with the FP32 solve's own error far below it."""
import numpy as np
import pytest

from oracle import encoder_ref as R
from tests.gpu_common import rel_l2, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda").contiguous()


def lib():
    from paper_2603_00035_amd import _lib as L
    return L


@pytest.mark.parametrize("B,Cin,Cout,relu", [(1, 4, 32, True), (3, 32, 5, False), (5, 37, 19, True),
                                            (2, 1, 1, False)])
def test_dense_forward_and_backward(B, Cin, Cout, relu):
    L = lib()
    rng = np.random.default_rng(B * 100 + Cin)
    x, W, b = rng.normal(size=(B, Cin)), rng.normal(size=(Cout, Cin)), rng.normal(size=Cout)
    x, W, b = (a.astype(np.float32).astype(np.float64) for a in (x, W, b))
    dy = rng.normal(size=(B, Cout)).astype(np.float32).astype(np.float64)
    say(f"[encoder] dense {B}x{Cin}->{Cout} relu={relu}")
    xd, Wd, bd, dyd = dev(x), dev(W), dev(b), dev(dy)
    y = torch.empty(B, Cout, device="cuda")
    st = L.stream_handle(torch.device("cuda"))
    L.check("dense", L.lib().eik_enc_dense(B, Cin, Cout, L.ptr(xd), L.ptr(Wd), L.ptr(bd), int(relu), L.ptr(y), st))
    ref = R.dense(x, W, b, relu)
    terms = np.abs(x) @ np.abs(W).T + np.abs(b)
    assert np.all(np.abs(y.cpu().numpy() - ref) <= (Cin + 1) * 2.0 ** -23 * terms + 1e-30)
    # backward: y from the kernel (the mask is the kernel's), gradients accumulate onto nonzero starts
    yo = y.cpu().numpy().astype(np.float64)
    dx = torch.empty(B, Cin, device="cuda")
    dW0, db0 = rng.normal(size=(Cout, Cin)).astype(np.float32), rng.normal(size=Cout).astype(np.float32)
    dW, db = dev(dW0), dev(db0)
    L.check("dense_bwd", L.lib().eik_enc_dense_backward(B, Cin, Cout, L.ptr(xd), L.ptr(Wd), L.ptr(y), int(relu),
                                                        L.ptr(dyd), L.ptr(dx), L.ptr(dW), L.ptr(db), st))
    rdx, rdW, rdb = R.dense_backward(x, W, yo, relu, dy)
    g = np.where(yo > 0, dy, 0.0) if relu else dy
    assert np.all(np.abs(dx.cpu().numpy() - rdx) <= Cout * 2.0 ** -23 * (np.abs(g) @ np.abs(W)) + 1e-30)
    assert np.all(np.abs(dW.cpu().numpy() - (dW0 + rdW)) <=
                  (B + 1) * 2.0 ** -23 * (np.abs(g).T @ np.abs(x) + np.abs(dW0)) + 1e-30)
    assert np.all(np.abs(db.cpu().numpy() - (db0 + rdb)) <= (B + 1) * 2.0 ** -23 * (np.abs(g).sum(0) + np.abs(db0)))


@pytest.mark.parametrize("dtype,B,n", [(torch.float32, 1, 4097), (torch.float64, 1, 1), (torch.float64, 1, 300 * 257),
                                       (torch.float32, 3, 1000), (torch.float64, 5, 257)])
def test_combine_forward_and_backward(dtype, B, n):
    """B scenes: base [B][5], local [5][B][n], M [B][3][n], omega [B][2][n];
    the oracle runs scene by scene."""
    L = lib()
    rng = np.random.default_rng(n + B)
    base = rng.normal(size=(B, 5)).astype(np.float32).astype(np.float64)
    local = rng.normal(size=(5, B, n)).astype(np.float32).astype(np.float64)
    alpha = 0.37
    say(f"[encoder] combine B={B} n={n} {dtype}")
    M = torch.empty(B, 3, n, dtype=dtype, device="cuda")
    om = torch.empty(B, 2, n, dtype=dtype, device="cuda")
    st = L.stream_handle(torch.device("cuda"))
    based, locald = dev(base), dev(local)  # referenced until the kernel has run
    L.check("combine", L.lib().eik_enc_combine(B, n, L.dtype_code(M), alpha, L.ptr(based), L.ptr(locald),
                                               L.ptr(M), L.ptr(om), st))
    got = np.concatenate([M.cpu().numpy(), om.cpu().numpy()], axis=1).astype(np.float64)
    # one rounding of the result, plus the product's rounding in the reference
    # (the kernel fuses the multiply-add), relative to the terms
    ulp = 2.0 ** -23 if dtype == torch.float32 else 2.0 ** -52
    for b in range(B):
        rM, rom = R.combine(base[b], local[:, b], alpha)
        ref = np.concatenate([rM, rom])
        terms = np.abs(base[b])[:, None] + alpha * np.abs(local[:, b])
        assert np.all(np.abs(got[b] - ref) <= ulp * np.abs(ref) + 2.0 ** -52 * terms + 1e-300)
    d = rng.normal(size=(B, 5, n))
    if dtype == torch.float32:
        d = d.astype(np.float32).astype(np.float64)
    dM, dom = dev(d[:, :3], dtype), dev(d[:, 3:], dtype)
    dl = torch.empty(5, B, n, device="cuda")
    dbase0 = rng.normal(size=(B, 5)).astype(np.float32)
    dbase = dev(dbase0)
    scratch = torch.empty(L.lib().eik_enc_scratch_bytes(B), dtype=torch.uint8, device="cuda")
    L.check("combine_bwd", L.lib().eik_enc_combine_backward(B, n, L.dtype_code(dM), alpha, L.ptr(dM), L.ptr(dom),
                                                            L.ptr(dl), L.ptr(dbase), L.ptr(scratch), st))
    dlg, dbg = dl.cpu().numpy(), dbase.cpu().numpy()
    for b in range(B):
        rdl, rdb = R.combine_backward(d[b, :3], d[b, 3:], alpha)
        assert np.array_equal(dlg[:, b], rdl.astype(np.float32))
        tot = dbase0[b] + rdb
        bound = n * 2.0 ** -52 * np.abs(d[b]).sum(1) + 2.0 ** -23 * np.abs(tot)
        assert np.all(np.abs(dbg[b] - tot) <= bound)


def make_case(seed, n):
    """Scene, oracle-made observations (FP64 solve on the hidden fields) and
    an encoder with its initial parameters; conv inputs padded to 16."""
    import oracle
    from paper_2603_00035_amd.encoder import Encoder
    from synthetic.covariates import scene
    from synthetic.fields import Problem
    sc = scene(seed, n=n)
    To, _, _ = oracle.forward(Problem(n, n, sc.h, sc.M, sc.omega, sc.src_idx, np.zeros(1)))
    mask = (To <= np.quantile(To, 0.7)).astype(np.uint8)
    enc = Encoder(device="cuda", seed=seed)
    return sc, To, mask, enc


@pytest.mark.parametrize("H,W", [(48, 48), (37, 70), (65, 23)])
def test_encoder_forward_matches_oracle(H, W):
    from paper_2603_00035_amd.encoder import CONV_NAMES
    sc, _, _, enc = make_case(21, 72)
    X = np.ascontiguousarray(sc.X[:, :H, :W])  # non-square and ragged grids from a larger scene
    # random, larger heads so that the spatial pathway carries weight in (M, omega)
    g = torch.Generator().manual_seed(5)
    for k in range(5):
        enc.params[f"head{k}.w"].copy_(torch.randn(16, generator=g) * 0.2)
    say(f"[encoder] forward {H}x{W}")
    enc.set_inputs(torch.tensor(X), torch.tensor(sc.y))
    M, om = enc.forward()
    P = {k: torch.tensor(v.numpy(), dtype=torch.float64) for k, v in enc.state_dict().items()}
    X16 = np.zeros((16, H, W))
    X16[:4] = X
    rM, rom = R.network(P, torch.tensor(X16), torch.tensor(sc.y), enc.alpha, CONV_NAMES)
    loc = enc.local.cpu().numpy()
    rloc = (np.concatenate([rM.detach().numpy(), rom.detach().numpy()]) -
            (P["g2.w"] @ torch.relu(P["g1.w"] @ torch.tensor(sc.y) + P["g1.b"]) + P["g2.b"]).detach().numpy()
            .reshape(5, 1, 1)) / enc.alpha
    e_loc = rel_l2([loc], [rloc])
    e_out = rel_l2([M.cpu().numpy(), om.cpu().numpy()], [rM.detach().numpy(), rom.detach().numpy()])
    say(f"[encoder] spatial pathway rel-L2 {e_loc:.2e}, (M, omega) rel-L2 {e_out:.2e}")
    assert e_loc <= 1e-2 and e_out <= 1e-3


def test_hybrid_gradient_matches_oracle():
    from paper_2603_00035_amd.encoder import CONV_NAMES, Trainer
    sc, To, mask, enc = make_case(22, 40)
    g = torch.Generator().manual_seed(6)
    for k in range(5):
        enc.params[f"head{k}.w"].copy_(torch.randn(16, generator=g) * 0.1)
    say("[encoder] hybrid gradient 40x40")
    tr = Trainer(enc, tol=0.0)
    src = torch.tensor(sc.src_idx, dtype=torch.int32, device="cuda")
    enc.zero_grads()
    T, s = tr.gradients(torch.tensor(sc.X), torch.tensor(sc.y), src, sc.h, dev(To), dev(mask, torch.uint8))
    params = {k: v.numpy().astype(np.float64) for k, v in enc.state_dict().items()}
    X16 = np.zeros((16, 40, 40))
    X16[:4] = sc.X
    go, Lo, _, _ = R.hybrid_gradient(params, X16, sc.y, enc.alpha, CONV_NAMES, sc.h, sc.src_idx, np.zeros(1), To,
                                     mask.astype(bool))
    Lg = float(s[0])
    say(f"[encoder] data term GPU {Lg:.6e} oracle {Lo:.6e}")
    assert abs(Lg - Lo) <= 1e-3 * Lo
    worst = 0.0
    for k in sorted(go):
        e = rel_l2([enc.grads[k].cpu().numpy()], [go[k]])
        worst = max(worst, e)
        say(f"[encoder]   d{k}: rel-L2 {e:.2e}")
        assert e <= 1e-2, k
    say(f"[encoder] worst parameter-gradient rel-L2 {worst:.2e}")


def test_batched_hybrid_gradient_is_the_sum_over_scenes():
    """Three scenes in one step (batched network, one batched solve and
    adjoint) against the sum of the oracle's per-scene hybrid gradients."""
    from paper_2603_00035_amd.encoder import CONV_NAMES, Trainer
    cases = [make_case(s, 40) for s in (31, 32, 33)]
    enc = cases[0][3]
    g = torch.Generator().manual_seed(7)
    for k in range(5):
        enc.params[f"head{k}.w"].copy_(torch.randn(16, generator=g) * 0.1)
    say("[encoder] batched hybrid gradient, 3 scenes of 40x40")
    tr = Trainer(enc, tol=0.0)
    enc.zero_grads()
    X = torch.stack([torch.tensor(c[0].X) for c in cases])
    y = torch.stack([torch.tensor(c[0].y) for c in cases])
    srcs = [torch.tensor(c[0].src_idx, dtype=torch.int32, device="cuda") for c in cases]
    To = dev(np.stack([c[1] for c in cases]))
    mk = dev(np.stack([c[2] for c in cases]), torch.uint8)
    T, s = tr.gradients_batch(X, y, srcs, cases[0][0].h, To, mk)
    params = {k: v.numpy().astype(np.float64) for k, v in enc.state_dict().items()}
    tot, Ltot = None, 0.0
    for sc, Tc, mask, _ in cases:
        X16 = np.zeros((16, 40, 40))
        X16[:4] = sc.X
        go, Lo, _, _ = R.hybrid_gradient(params, X16, sc.y, enc.alpha, CONV_NAMES, sc.h, sc.src_idx, np.zeros(1), Tc,
                                         mask.astype(bool))
        tot = go if tot is None else {k: tot[k] + go[k] for k in tot}
        Ltot += Lo
    say(f"[encoder] data term GPU {float(s[0]):.6e} oracle {Ltot:.6e}")
    assert abs(float(s[0]) - Ltot) <= 1e-3 * Ltot
    worst = max(rel_l2([enc.grads[k].cpu().numpy()], [tot[k]]) for k in tot)
    say(f"[encoder] worst parameter-gradient rel-L2 {worst:.2e}")
    assert worst <= 1e-2


def test_training_lowers_the_loss():
    from paper_2603_00035_amd.encoder import Trainer, correlation
    sc, To, mask, enc = make_case(23, 64)
    tr = Trainer(enc, lr=3e-3)
    src = torch.tensor(sc.src_idx, dtype=torch.int32, device="cuda")
    scn = {"X": torch.tensor(sc.X), "y": torch.tensor(sc.y), "src": src, "h": sc.h, "T_obs": dev(To),
           "mask": dev(mask, torch.uint8)}
    losses = [float(tr.step(scn)[0]) for _ in range(60)]
    T, _ = tr.predict(scn["X"], scn["y"], src, sc.h)
    r = correlation(T, scn["T_obs"], scn["mask"])
    say(f"[encoder] loss {losses[0]:.4e} -> {losses[-1]:.4e}, correlation {r:.3f}")
    assert losses[-1] < 0.5 * losses[0]
    assert all(np.isfinite(losses))
