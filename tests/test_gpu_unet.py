"""The warm-start network's BF16 MFMA kernels through their C ABI, against the
float64 oracle layers on the same bf16-rounded operands. Tolerance from the
arithmetic: bf16 x bf16 products are exact in FP32, the FP32 sum of K terms is
within K 2^-24 sum|terms|, and a bf16 output adds one rounding (2^-9 relative)."""
import ctypes

import numpy as np
import pytest

from oracle import unet_ref as U
from tests.gpu_common import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def lib():
    from paper_2603_00035_amd import unet
    return unet._bind()


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def st():
    from paper_2603_00035_amd import _lib as L
    return L.stream_handle(torch.device("cuda"))


_KEEP = []  # device inputs stay referenced until the test ends (a temporary's memory could be reused)


def to_dev_bf16(x):
    t = torch.tensor(U.bf16_bits(x).view(np.int16), device="cuda")
    _KEEP.append(t)
    return t


def to_dev(x):
    t = torch.tensor(x, device="cuda")
    _KEEP.append(t)
    return t


@pytest.fixture(autouse=True)
def _release_inputs():
    yield
    torch.cuda.synchronize()
    _KEEP.clear()


def from_dev_bf16(t, shape):
    return U.from_bits(t.cpu().numpy().view(np.uint16)).reshape(shape)


def check(got, ref, absterms, K, out_bf16=True):
    tol = K * 2.0 ** -23 * absterms + (2.0 ** -8 * np.abs(ref) if out_bf16 else 0) + 1e-30
    bad = np.abs(got - ref) > tol
    assert not bad.any(), f"{bad.sum()} elements off; worst {np.max(np.abs(got - ref) / tol):.2f}x tol"


@pytest.mark.parametrize("B,H,W,Cin,Cout,relu", [(2, 16, 32, 16, 16, True), (1, 8, 64, 32, 64, False),
                                                (3, 32, 16, 64, 128, True), (1, 5, 7, 16, 48, True)])
def test_conv3_forward(B, H, W, Cin, Cout, relu):
    rng = np.random.default_rng(B * 100 + Cout)
    x = U.bf16_round(rng.standard_normal((B, H, W, Cin)))
    w = U.bf16_round(rng.standard_normal((9, Cout, Cin)) * 0.2)
    bias = rng.standard_normal(Cout).astype(np.float32)
    say(f"[unet] conv3 {B}x{H}x{W} {Cin}->{Cout}")
    yd = torch.zeros(B * H * W * Cout, dtype=torch.int16, device="cuda")
    bd = torch.tensor(bias, device="cuda")
    rc = lib().eiku_conv_fwd(0, B, H, W, P(to_dev_bf16(x)), Cin, 0, Cin, P(to_dev_bf16(w)), P(bd), int(relu),
                             P(yd), Cout, 0, Cout, st())
    assert rc == 0
    got = from_dev_bf16(yd, (B, H, W, Cout))
    ref = U.conv3(x, w, bias.astype(np.float64), relu)
    absterms = U.conv3(np.abs(x), np.abs(w)) + np.abs(bias)
    check(got, ref, absterms, 9 * Cin + 1)


def test_channel_slices_up2_down2_and_gradients():
    rng = np.random.default_rng(5)
    B, H, W, Cin, Cout = 2, 8, 16, 32, 16
    x = U.bf16_round(rng.standard_normal((B, H, W, Cin)))
    w = U.bf16_round(rng.standard_normal((4, Cout, Cin)) * 0.3)
    say("[unet] up2 into a channel slice, down2, weight gradients")
    # up2 writes channels 16..31 of a 32-channel buffer at twice the resolution
    yd = torch.zeros(B * 2 * H * 2 * W * 32, dtype=torch.int16, device="cuda")
    assert lib().eiku_conv_fwd(1, B, H, W, P(to_dev_bf16(x)), Cin, 0, Cin, P(to_dev_bf16(w)), None, 0, P(yd), 32, 16,
                               Cout, st()) == 0
    got = from_dev_bf16(yd, (B, 2 * H, 2 * W, 32))
    ref = U.up2(x, w)
    check(got[..., 16:], ref, U.up2(np.abs(x), np.abs(w)), Cin)
    assert np.all(got[..., :16] == 0)
    # down2 (data gradient of up2) from a channel slice
    g = U.bf16_round(rng.standard_normal((B, 2 * H, 2 * W, Cout)))
    gbuf = np.zeros((B, 2 * H, 2 * W, 32))
    gbuf[..., 16:] = g
    wt = U.bf16_round(w.transpose(0, 2, 1).copy())
    dd = torch.zeros(B * H * W * Cin, dtype=torch.int16, device="cuda")
    assert lib().eiku_conv_fwd(2, B, H, W, P(to_dev_bf16(gbuf)), 32, 16, Cout, P(to_dev_bf16(wt)), None, 0, P(dd),
                               Cin, 0, Cin, st()) == 0
    check(from_dev_bf16(dd, (B, H, W, Cin)), U.down2(g, wt), U.down2(np.abs(g), np.abs(wt)), 4 * Cout)
    # weight gradient of up2
    dw = torch.zeros(4 * Cout * Cin, dtype=torch.float32, device="cuda")
    assert lib().eiku_conv_wgrad(1, B, H, W, P(to_dev_bf16(x)), Cin, 0, Cin, P(to_dev_bf16(gbuf)), 32, 16, Cout,
                                 P(dw), st()) == 0
    npix = B * H * W
    check(dw.cpu().numpy().reshape(4, Cout, Cin), U.up2_wgrad(x, g), U.up2_wgrad(np.abs(x), np.abs(g)), npix,
          out_bf16=False)
    # weight gradient of conv3
    x3 = U.bf16_round(rng.standard_normal((B, H, W, 16)))
    g3 = U.bf16_round(rng.standard_normal((B, H, W, 32)))
    dw3 = torch.zeros(9 * 32 * 16, dtype=torch.float32, device="cuda")
    assert lib().eiku_conv_wgrad(0, B, H, W, P(to_dev_bf16(x3)), 16, 0, 16, P(to_dev_bf16(g3)), 32, 0, 32, P(dw3),
                                 st()) == 0
    check(dw3.cpu().numpy().reshape(9, 32, 16), U.conv3_wgrad(x3, g3), U.conv3_wgrad(np.abs(x3), np.abs(g3)), npix,
          out_bf16=False)


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(1, 5, 9, 128, 64), (2, 12, 40, 64, 32), (3, 16, 32, 32, 16)])
def test_up2_and_down2_ragged_multi_slice(B, H, W, Cin, Cout):
    """The transposed convolution over several 32-channel slices and all four
    taps in one workgroup, and its data gradient over 16-channel slices, on
    grids that are not multiples of the 8 x 32 tile."""
    rng = np.random.default_rng(H * W + Cin)
    x = U.bf16_round(rng.standard_normal((B, H, W, Cin)))
    w = U.bf16_round(rng.standard_normal((4, Cout, Cin)) * 0.2)
    bias = rng.standard_normal(Cout).astype(np.float32)
    say(f"[unet] up2/down2 {B}x{H}x{W} {Cin}<->{Cout}")
    yd = torch.zeros(B * 4 * H * W * Cout, dtype=torch.int16, device="cuda")
    assert lib().eiku_conv_fwd(1, B, H, W, P(to_dev_bf16(x)), Cin, 0, Cin, P(to_dev_bf16(w)), P(to_dev(bias)), 1,
                               P(yd), Cout, 0, Cout, st()) == 0
    ref = np.maximum(U.up2(x, w) + bias, 0.0)
    check(from_dev_bf16(yd, (B, 2 * H, 2 * W, Cout)), ref, U.up2(np.abs(x), np.abs(w)) + np.abs(bias), Cin + 1)
    g = U.bf16_round(rng.standard_normal((B, 2 * H, 2 * W, Cout)))
    wt = U.bf16_round(w.transpose(0, 2, 1).copy())
    dd = torch.zeros(B * H * W * Cin, dtype=torch.int16, device="cuda")
    assert lib().eiku_conv_fwd(2, B, H, W, P(to_dev_bf16(g)), Cout, 0, Cout, P(to_dev_bf16(wt)), None, 0, P(dd),
                               Cin, 0, Cin, st()) == 0
    check(from_dev_bf16(dd, (B, H, W, Cin)), U.down2(g, wt), U.down2(np.abs(g), np.abs(wt)), 4 * Cout)


@pytest.mark.parametrize("B,H,W,Cin,Cout,xs,dys", [(1, 5, 7, 16, 16, (16, 0), (16, 0)),
                                                   (2, 24, 40, 64, 128, (64, 0), (128, 0)),
                                                   (3, 20, 36, 32, 16, (64, 32), (32, 16)),
                                                   (16, 256, 256, 16, 16, (16, 0), (16, 0))])
def test_conv3_weight_gradient(B, H, W, Cin, Cout, xs, dys):
    """The 3x3 weight gradient: ragged tiles, 32 x 32 channel blocks, channel
    slices of wider buffers, and (at 16 x 256^2) workgroups that run over
    several pixel tiles before their atomics."""
    rng = np.random.default_rng(B + H + Cin)
    x = U.bf16_round(rng.standard_normal((B, H, W, Cin)))
    g = U.bf16_round(rng.standard_normal((B, H, W, Cout)))
    xb = np.zeros((B, H, W, xs[0]))
    xb[..., xs[1]:xs[1] + Cin] = x
    gb = np.zeros((B, H, W, dys[0]))
    gb[..., dys[1]:dys[1] + Cout] = g
    say(f"[unet] conv3 wgrad {B}x{H}x{W} {Cin}->{Cout}, x slice {xs}, dy slice {dys}")
    dw = torch.zeros(9 * Cout * Cin, dtype=torch.float32, device="cuda")
    assert lib().eiku_conv_wgrad(0, B, H, W, P(to_dev_bf16(xb)), xs[0], xs[1], Cin, P(to_dev_bf16(gb)), dys[0],
                                 dys[1], Cout, P(dw), st()) == 0
    check(dw.cpu().numpy().reshape(9, Cout, Cin), U.conv3_wgrad(x, g), U.conv3_wgrad(np.abs(x), np.abs(g)),
          B * H * W, out_bf16=False)


@pytest.mark.parametrize("B,H,W,Ca,Cb,Cout,pad", [(2, 16, 40, 16, 16, 16, 0), (1, 9, 33, 32, 32, 32, 8),
                                                  (2, 8, 32, 64, 64, 64, 0), (1, 5, 7, 16, 48, 16, 16)])
def test_conv3_two_sources_equal_one_concatenated_buffer(B, H, W, Ca, Cb, Cout, pad):
    """The _cat forms read the concatenation [xa | xb] from two buffers (each a
    channel slice of a wider one when pad > 0). The forward meets the oracle's
    arithmetic bound, and equals the one-buffer convolution of the
    concatenation bit for bit when both take the same K slices (32 channels
    when both halves are multiples of 32 or neither form can, else the two
    sources go in 16-channel slices and only the rounding order differs). The
    weight gradient meets the oracle's bound."""
    rng = np.random.default_rng(B + H + Ca + Cb)
    Cin = Ca + Cb
    xa = U.bf16_round(rng.standard_normal((B, H, W, Ca)))
    xb = U.bf16_round(rng.standard_normal((B, H, W, Cb)))
    x = np.concatenate([xa, xb], -1)
    w = U.bf16_round(rng.standard_normal((9, Cout, Cin)) * 0.2)
    bias = rng.standard_normal(Cout).astype(np.float32)
    g = U.bf16_round(rng.standard_normal((B, H, W, Cout)))

    def slab(v, C):  # v as channels pad .. pad+C-1 of a wider buffer
        out = np.zeros(v.shape[:-1] + (C + 2 * pad,))
        out[..., pad:pad + C] = v
        return to_dev_bf16(out)

    da, db = slab(xa, Ca), slab(xb, Cb)
    say(f"[unet] conv3 of [{Ca} | {Cb}] channels, {B}x{H}x{W} -> {Cout}, slice offset {pad}")
    bd = to_dev(bias)
    y_cat = torch.zeros(B * H * W * Cout, dtype=torch.int16, device="cuda")
    y_one = torch.zeros_like(y_cat)
    wd = to_dev_bf16(w)
    assert lib().eiku_conv_fwd_cat(B, H, W, P(da), Ca + 2 * pad, pad, Ca, P(db), Cb + 2 * pad, pad, Cb, P(wd), P(bd), 1,
                                   P(y_cat), Cout, 0, Cout, st()) == 0
    assert lib().eiku_conv_fwd(0, B, H, W, P(to_dev_bf16(x)), Cin, 0, Cin, P(wd), P(bd), 1, P(y_one), Cout, 0, Cout,
                               st()) == 0
    same_k = (Ca % 32 == 0 and Cb % 32 == 0) or Cin % 32 != 0
    if same_k:
        assert torch.equal(y_cat.cpu(), y_one.cpu())
    ref = U.conv3(x, w, bias.astype(np.float64), True)
    absterms = U.conv3(np.abs(x), np.abs(w)) + np.abs(bias)
    check(from_dev_bf16(y_cat, (B, H, W, Cout)), ref, absterms, 9 * Cin + 1)
    check(from_dev_bf16(y_one, (B, H, W, Cout)), ref, absterms, 9 * Cin + 1)
    dw = torch.zeros(9 * Cout * Cin, dtype=torch.float32, device="cuda")
    assert lib().eiku_conv_wgrad_cat(B, H, W, P(da), Ca + 2 * pad, pad, Ca, P(db), Cb + 2 * pad, pad, Cb,
                                     P(to_dev_bf16(g)), Cout, 0, Cout, P(dw), st()) == 0
    check(dw.cpu().numpy().reshape(9, Cout, Cin), U.conv3_wgrad(x, g), U.conv3_wgrad(np.abs(x), np.abs(g)),
          B * H * W, out_bf16=False)


@pytest.mark.parametrize("mode,Cin,Cout,cat", [(0, 16, 16, False), (0, 32, 32, True), (1, 32, 16, False)])
def test_multi_tile_workgroups_equal_single_image_launches(mode, Cin, Cout, cat):
    """Launches of 32 768 pixel tiles or more give each workgroup two tiles (the
    second tile's loads in flight while the first is computed). 111 grids of
    260 x 264 make 32 967 tiles, ragged in both directions, the last workgroup
    with one tile: the outputs of sampled grids equal those of launches over
    that grid alone (one tile per workgroup) bit for bit, and the first grid's
    meet the oracle's bound."""
    B, H, W = 111, 260, 264
    say(f"[unet] mode {mode} {Cin}->{Cout}{' from two buffers' if cat else ''}, {B}x{H}x{W}: two tiles per workgroup")
    gen = torch.Generator(device="cuda").manual_seed(Cin + Cout + mode)
    x = torch.randn(B, H, W, Cin, device="cuda", generator=gen).to(torch.bfloat16).view(torch.int16)
    rng = np.random.default_rng(Cin * Cout)
    taps = 9 if mode == 0 else 4
    w = U.bf16_round(rng.standard_normal((taps, Cout, Cin)) * 0.2)
    bias = rng.standard_normal(Cout).astype(np.float32)
    wd, bd = to_dev_bf16(w), to_dev(bias)
    Ho, Wo = (H, W) if mode == 0 else (2 * H, 2 * W)
    h = Cin // 2
    xa, xb = (x[..., :h].contiguous(), x[..., h:].contiguous()) if cat else (None, None)

    def run(sel, n):
        y = torch.zeros(n, Ho, Wo, Cout, dtype=torch.int16, device="cuda")
        if cat:
            rc = lib().eiku_conv_fwd_cat(n, H, W, P(xa[sel]), h, 0, h, P(xb[sel]), h, 0, h, P(wd), P(bd), 1, P(y),
                                         Cout, 0, Cout, st())
        else:
            rc = lib().eiku_conv_fwd(mode, n, H, W, P(x[sel]), Cin, 0, Cin, P(wd), P(bd), int(mode == 0), P(y), Cout,
                                     0, Cout, st())
        assert rc == 0
        return y

    y_all = run(slice(0, B), B)
    for g in (0, 55, B - 1):
        y_one = run(slice(g, g + 1), 1)
        assert torch.equal(y_all[g].cpu(), y_one[0].cpu()), f"grid {g}"
    x0 = U.from_bits(x[0].cpu().numpy().view(np.uint16)).reshape(H, W, Cin)[None]
    got = from_dev_bf16(y_all[0], (1, Ho, Wo, Cout))
    if mode == 0:
        ref = U.conv3(x0, w, bias.astype(np.float64), True)
        check(got, ref, U.conv3(np.abs(x0), np.abs(w)) + np.abs(bias), 9 * Cin + 1)
    else:
        ref = U.up2(x0, w, bias.astype(np.float64))
        check(got, ref, U.up2(np.abs(x0), np.abs(w)) + np.abs(bias), Cin + 1)


def test_weight_prep_mirrors_taps_for_the_data_gradient():
    """conv3 with the prepared backward weights is the adjoint of conv3."""
    rng = np.random.default_rng(6)
    Cout, Cin = 32, 16
    w32 = rng.standard_normal((9, Cout, Cin)).astype(np.float32)
    wf = torch.zeros(9 * Cout * Cin, dtype=torch.int16, device="cuda")
    wb = torch.zeros(9 * Cout * Cin, dtype=torch.int16, device="cuda")
    assert lib().eiku_prep_weights(0, 9, Cout, Cin, Cin, P(to_dev(w32)), P(wf), P(wb), st()) == 0
    wfr = from_dev_bf16(wf, (9, Cout, Cin))
    wbr = from_dev_bf16(wb, (9, Cin, Cout))
    assert np.array_equal(wfr, U.bf16_round(w32))
    assert np.array_equal(wbr, wfr[::-1].transpose(0, 2, 1))


def test_pool_head_features_and_adam():
    rng = np.random.default_rng(7)
    B, H, W, C = 2, 8, 8, 16
    x = U.bf16_round(rng.standard_normal((B, 2 * H, 2 * W, C)))
    yd = torch.zeros(B * H * W * C, dtype=torch.int16, device="cuda")
    xd = to_dev_bf16(x)
    assert lib().eiku_maxpool_fwd(B, H, W, P(xd), C, 0, P(yd), C, 0, C, st()) == 0
    assert np.array_equal(from_dev_bf16(yd, (B, H, W, C)), U.maxpool(x))
    dy = U.bf16_round(rng.standard_normal((B, H, W, C)))
    dxd = torch.zeros(B * 2 * H * 2 * W * C, dtype=torch.int16, device="cuda")
    assert lib().eiku_maxpool_bwd(B, H, W, P(xd), C, 0, P(to_dev_bf16(dy)), C, 0, P(dxd), C, 0, C, st()) == 0
    assert np.array_equal(from_dev_bf16(dxd, x.shape), U.maxpool_bwd(x, dy))
    hw = rng.standard_normal(16).astype(np.float32)
    hb = np.array([0.5], np.float32)
    xh = U.bf16_round(rng.standard_normal((B * H * W, 16)))
    out = torch.zeros(B * H * W, device="cuda")
    assert lib().eiku_head_fwd(B * H * W, P(to_dev_bf16(xh)), 16, 0, 16, P(to_dev(hw)),
                               P(to_dev(hb)), P(out), st()) == 0
    ref = U.head(xh, hw.astype(np.float64), 0.5)
    assert np.allclose(out.cpu().numpy(), ref, rtol=1e-5, atol=1e-5)
    # Adam on a quadratic: one step moves every parameter by lr against the gradient sign
    p = torch.ones(100, device="cuda")
    g = torch.linspace(-1, 1, 100, device="cuda")
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    gs = g.clone()
    assert lib().eiku_adam(100, P(p), P(g), P(m), P(v), 0.01, 0.9, 0.999, 1e-8, 1, st()) == 0
    exp = 1 - 0.01 * gs / (gs.abs() + 1e-8)
    assert torch.allclose(p, exp, atol=1e-6) and torch.all(g == 0)


@pytest.mark.parametrize("C,cs,co", [(32, 64, 32), (12, 12, 0), (16, 48, 8)])
def test_pool_and_head_on_slices_and_odd_channel_counts(C, cs, co):
    """Max pooling and the head on channel slices of wider buffers and on
    channel counts that are not multiples of 8 (the 16-byte and the per-channel
    kernels), against their definitions."""
    rng = np.random.default_rng(C + cs)
    B, H, W = 2, 6, 10
    x = U.bf16_round(rng.standard_normal((B, 2 * H, 2 * W, C)))
    xb = np.zeros((B, 2 * H, 2 * W, cs))
    xb[..., co:co + C] = x
    yd = torch.zeros(B * H * W * cs, dtype=torch.int16, device="cuda")
    assert lib().eiku_maxpool_fwd(B, H, W, P(to_dev_bf16(xb)), cs, co, P(yd), cs, co, C, st()) == 0
    got = from_dev_bf16(yd, (B, H, W, cs))
    assert np.array_equal(got[..., co:co + C], U.maxpool(x))
    assert np.all(got[..., :co] == 0) and np.all(got[..., co + C:] == 0)
    if C <= 16:
        hw = rng.standard_normal(C).astype(np.float32)
        xh = U.bf16_round(rng.standard_normal((B * H * W, C)))
        xhb = np.zeros((B * H * W, cs))
        xhb[:, co:co + C] = xh
        out = torch.zeros(B * H * W, device="cuda")
        assert lib().eiku_head_fwd(B * H * W, P(to_dev_bf16(xhb)), cs, co, C, P(to_dev(hw)),
                                   P(to_dev(np.array([0.25], np.float32))), P(out), st()) == 0
        ref = U.head(xh, hw.astype(np.float64), 0.25)
        assert np.allclose(out.cpu().numpy(), ref, rtol=1e-5, atol=1e-5)


def test_features_are_the_rounded_inputs_and_the_source_distance():
    rng = np.random.default_rng(11)
    B, H, W = 3, 16, 24
    M = rng.uniform(0.5, 2, (B, 3, H, W)).astype(np.float32)
    om = rng.uniform(-0.3, 0.3, (B, 2, H, W)).astype(np.float32)
    src = np.array([[5, 100, -1], [0, -1, -1], [H * W - 1, 37, 200]], np.int32)
    h = np.array([0.1, 0.05, 0.2], np.float32)
    x = torch.zeros(B * H * W * 16, dtype=torch.int16, device="cuda")
    dist = torch.zeros(B * H * W, device="cuda")
    assert lib().eiku_features(B, H, W, P(to_dev(M)), P(to_dev(om)), P(to_dev(src)), 3, P(to_dev(h)), P(x),
                               P(dist), st()) == 0
    got = from_dev_bf16(x, (B, H, W, 16))
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for b in range(B):
        s = [c for c in src[b] if c >= 0]
        d2 = np.min([(ii - c % W) ** 2 + (jj - c // W) ** 2 for c in s], axis=0).astype(np.float32)
        d = np.sqrt(d2) * h[b]  # FP32 throughout, as the kernel computes it
        assert np.array_equal(dist.cpu().numpy().reshape(B, H, W)[b], d)
        want = np.stack([M[b, 0], M[b, 1], M[b, 2], om[b, 0], om[b, 1], d], -1)
        assert np.array_equal(got[b, ..., :6], U.bf16_round(want))
        assert np.all(got[b, ..., 6:] == 0)


def test_network_forward_matches_the_oracle_composition_of_its_layers():
    """The whole forward (17 convolutions, 3 poolings, the head) against the
    oracle's layers composed in float64, each stored activation rounded to
    bfloat16 as the kernels store it, with the skip tensor first in every
    concatenation. FP32 accumulation against float64 flips a bf16 rounding now
    and then (one bf16 step, 2^-8 relative, of an element); the prediction's
    relative L2 difference stays orders of magnitude below 1e-2, which a
    mis-wired layer (swapped concatenation halves, a wrong pooling source)
    exceeds by far."""
    from paper_2603_00035_amd.unet import LAYERS, UNet
    net = UNet(seed=11)
    B, H, W = 2, 40, 48
    rng = np.random.default_rng(12)
    for name, *_ in LAYERS:
        net.params[name + ".b"].copy_(torch.tensor(rng.standard_normal(net.params[name + ".b"].numel()) * 0.1))
    b = net._layout(B, H, W)
    x0 = np.zeros((B, H, W, 16))
    x0[..., :6] = U.bf16_round(rng.uniform(-1, 1, (B, H, W, 6)))
    b["x0"].copy_(torch.tensor(U.bf16_bits(x0).view(np.int16).reshape(-1), device="cuda"))
    say(f"[unet] whole forward {B}x{H}x{W} against the oracle's layers")
    pred = net.forward(B, H, W).cpu().numpy().astype(np.float64).reshape(B, H, W)

    P_ = {k: v.cpu().numpy().astype(np.float64) for k, v in net.params.items()}
    R = U.bf16_round

    def conv(name, x, relu=True):
        return R(U.conv3(x, R(P_[name + ".w"]), P_[name + ".b"], relu))

    def up(name, x):
        return R(U.up2(x, R(P_[name + ".w"]), P_[name + ".b"]))

    s0 = conv("e0b", conv("e0a", x0))
    s1 = conv("e1b", conv("e1a", U.maxpool(s0)))
    s2 = conv("e2b", conv("e2a", U.maxpool(s1)))
    bb = conv("bb", conv("ba", U.maxpool(s2)))
    d2 = conv("d2b", conv("d2a", np.concatenate([s2, up("u2", bb)], -1)))
    d1 = conv("d1b", conv("d1a", np.concatenate([s1, up("u1", d2)], -1)))
    d0 = conv("d0b", conv("d0a", np.concatenate([s0, up("u0", d1)], -1)))
    ref = U.head(d0, P_["head.w"], P_["head.b"][0])
    r = np.linalg.norm(pred - ref) / np.linalg.norm(ref)
    say(f"  prediction rel L2 {r:.2e}")
    assert r <= 1e-2


def test_network_gradient_matches_finite_differences_of_its_loss():
    """End to end: the backward pass of the whole network (all kernels) agrees
    with central differences of its own forward loss on a few parameters."""
    from paper_2603_00035_amd.unet import UNet
    from paper_2603_00035_amd import _lib as L
    net = UNet(seed=3)
    B, H, W = 1, 32, 32
    rng = np.random.default_rng(8)
    M = torch.tensor(rng.uniform(0.5, 2, (B, 3, H, W)), dtype=torch.float32, device="cuda")
    M[:, 1] = 0.1
    om = torch.tensor(rng.uniform(-0.2, 0.2, (B, 2, H, W)), dtype=torch.float32, device="cuda")
    src = torch.tensor([[5 * W + 7, -1, -1, -1]], dtype=torch.int32, device="cuda")
    hv = torch.full((B,), 1.0 / 31, device="cuda")
    net.features(M, om, src, hv)
    target = torch.rand(B * H * W, device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))

    def loss():
        pred = net.forward(B, H, W)
        return float(((pred - target) ** 2).mean())

    pred = net.forward(B, H, W)
    lbuf = torch.zeros(1, device="cuda")
    net.lib.eiku_mse(pred.numel(), P(pred), P(target), P(lbuf), P(net._bufs["g_pred"]), st())
    net.zero_grads()
    net.backward(B, H, W)
    torch.cuda.synchronize()
    def central(p, idx, eps):
        old = float(p.view(-1)[idx])
        p.view(-1)[idx] = old + eps
        net.refresh_weights()
        lp = loss()
        p.view(-1)[idx] = old - eps
        net.refresh_weights()
        lm = loss()
        p.view(-1)[idx] = old
        net.refresh_weights()
        return (lp - lm) / (2 * eps)

    # each tensor at its largest-gradient entry: small entries are sums with
    # heavy cancellation, where BF16 rounding of the backward dominates
    for key in ["head.b", "d0b.b", "bb.b", "e1a.b", "u0.b"]:
        p = net.params[key]
        idx = int(net.grads[key].view(-1).abs().argmax())
        # the bf16 activations make the loss a step function at fine scales:
        # the spread of two step sizes measures that noise in the difference
        fd1, fd2 = central(p, idx, 0.05), central(p, idx, 0.025)
        an = float(net.grads[key].view(-1)[idx])
        say(f"  {key}[{idx}]: analytic {an:.4e} fd {fd1:.4e} / {fd2:.4e}")
        assert abs(an - fd1) <= 3 * abs(fd1 - fd2) + 0.1 * abs(fd1) + 1e-5


@pytest.mark.parametrize("npix,cs,co,C", [(4096, 64, 0, 64), (65536 + 37, 32, 16, 16), (1000, 128, 0, 128),
                                          (777, 48, 0, 48), (5, 16, 0, 16)])
def test_bias_gradient_matches_the_sum(npix, cs, co, C):
    """db[c] += sum_p dy(p, c) over a channel slice, accumulated onto a
    nonzero start; FP32 partial sums in any order are within
    npix 2^-24 sum|dy| of the exact sum."""
    rng = np.random.default_rng(npix + C)
    dy = U.bf16_round(rng.standard_normal((npix, cs)))
    db0 = rng.standard_normal(C).astype(np.float32)
    db = torch.tensor(db0, device="cuda")
    say(f"[unet] bias grad npix={npix} slice {co}:{co + C} of {cs}")
    assert lib().eiku_bias_grad(npix, P(to_dev_bf16(dy)), cs, co, C, P(db), st()) == 0
    ref = db0 + dy[:, co:co + C].sum(0)
    tol = (npix + 1) * 2.0 ** -23 * (np.abs(dy[:, co:co + C]).sum(0) + np.abs(db0)) + 1e-30
    assert np.all(np.abs(db.cpu().numpy() - ref) <= tol)


@pytest.mark.parametrize("npix,C", [(4096, 16), (65536 * 2 + 13, 16), (300, 7)])
def test_head_backward_matches_its_definition(npix, C):
    """dx(p, c) = w[c] g(p) (bfloat16), dw[c] += sum_p g(p) x(p, c),
    db += sum_p g(p)."""
    rng = np.random.default_rng(npix * 3 + C)
    x = U.bf16_round(rng.standard_normal((npix, 16)))
    w = rng.standard_normal(C).astype(np.float32)
    g = rng.standard_normal(npix).astype(np.float32)
    dx = torch.zeros(npix * 16, dtype=torch.int16, device="cuda")
    dw0 = rng.standard_normal(C).astype(np.float32)
    dw, dbt = torch.tensor(dw0, device="cuda"), torch.zeros(1, device="cuda")
    say(f"[unet] head backward npix={npix} C={C}")
    assert lib().eiku_head_bwd(npix, P(to_dev_bf16(x)), 16, 0, C, P(to_dev(w)), P(to_dev(g)), P(dx), 16, 0, P(dw),
                               P(dbt), st()) == 0
    dxg = from_dev_bf16(dx, (npix, 16))[:, :C]
    ref_dx = U.bf16_round(g.astype(np.float64)[:, None] * w.astype(np.float64)[None, :])
    assert np.array_equal(dxg, ref_dx)
    gx = g.astype(np.float64)[:, None] * x[:, :C]
    ref_dw = dw0 + gx.sum(0)
    assert np.all(np.abs(dw.cpu().numpy() - ref_dw) <= (npix + 1) * 2.0 ** -23 * (np.abs(gx).sum(0) + np.abs(dw0)))
    assert abs(float(dbt.cpu()[0]) - g.astype(np.float64).sum()) <= (npix + 1) * 2.0 ** -23 * np.abs(g).sum()
