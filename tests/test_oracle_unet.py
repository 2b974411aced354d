"""Pins of the network-layer oracle against independent definitions: scipy's
2-D correlation, element loops on tiny inputs, adjoint identities between a
layer and its gradients, and torch's bfloat16 rounding. CPU only."""
import numpy as np
import pytest
import scipy.signal

from oracle import unet_ref as U


def test_bf16_rounding_matches_torch():
    import torch
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10.0 ** np.random.default_rng(1).uniform(
        -5, 5, 10000).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16_round(x), ref)
    assert np.array_equal(U.from_bits(U.bf16_bits(x)), ref)


def test_conv3_matches_scipy_correlate():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((9, 4, 3))
    y = U.conv3(x, w)
    for b in range(2):
        for co in range(4):
            acc = np.zeros((7, 9))
            for ci in range(3):
                k = w[:, co, ci].reshape(3, 3)  # k[dy+1, dx+1]
                acc += scipy.signal.correlate2d(x[b, :, :, ci], k, mode="same", boundary="fill")
            assert np.allclose(y[b, :, :, co], acc, atol=1e-12)


def test_up2_and_maxpool_by_element_loops():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 3, 2, 2))
    w = rng.standard_normal((4, 3, 2))
    y = U.up2(x, w)
    for yy in range(3):
        for xx in range(2):
            for a in range(2):
                for c in range(2):
                    assert np.allclose(y[0, 2 * yy + a, 2 * xx + c], w[2 * a + c] @ x[0, yy, xx])
    z = rng.standard_normal((1, 4, 6, 2))
    m = U.maxpool(z)
    for yy in range(2):
        for xx in range(3):
            assert np.allclose(m[0, yy, xx], z[0, 2 * yy:2 * yy + 2, 2 * xx:2 * xx + 2].reshape(4, 2).max(axis=0))


def test_adjoint_identities():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 6, 8, 3))
    w = rng.standard_normal((9, 5, 3))
    g = rng.standard_normal((2, 6, 8, 5))
    # data gradient of conv3 = conv3 with mirrored taps and swapped channels
    wb = w[::-1].transpose(0, 2, 1)
    assert np.sum(U.conv3(x, w) * g) == pytest.approx(np.sum(x * U.conv3(g, wb)), rel=1e-12)
    # weight gradient: <conv3_w(x), g> = <w, wgrad(x, g)>
    assert np.sum(U.conv3(x, w) * g) == pytest.approx(np.sum(w * U.conv3_wgrad(x, g)), rel=1e-12)
    wu = rng.standard_normal((4, 5, 3))
    gu = rng.standard_normal((2, 12, 16, 5))
    assert np.sum(U.up2(x, wu) * gu) == pytest.approx(np.sum(x * U.down2(gu, wu.transpose(0, 2, 1))), rel=1e-12)
    assert np.sum(U.up2(x, wu) * gu) == pytest.approx(np.sum(wu * U.up2_wgrad(x, gu)), rel=1e-12)
    # maxpool backward is the adjoint of selecting the first maximum
    z = rng.standard_normal((1, 4, 4, 2))
    dz = rng.standard_normal((1, 2, 2, 2))
    assert np.sum(U.maxpool(z) * dz) == pytest.approx(np.sum(z * U.maxpool_bwd(z, dz)), rel=1e-12)
