"""The gradient-stability check's noise fields (CPU): unit variance per metric
plane, independent per node, or spatially correlated over the requested
number of nodes."""
import numpy as np
import torch

from paper_2603_00035_amd import gradcheck as C


def make(n=64, seed=0):
    c = C.Check.__new__(C.Check)
    c.n, c.dev, c.rng = n, torch.device("cpu"), np.random.default_rng(seed)
    c.M = torch.zeros(3, n, n, dtype=torch.float64)
    return c


def lag1(Z):
    return float(np.corrcoef(Z[:, :, :-1].ravel(), Z[:, :, 1:].ravel())[0, 1])


def test_independent_noise_has_unit_variance_and_no_spatial_correlation():
    Z = make().noise_field(None).numpy()
    assert np.allclose(Z.std(axis=(1, 2)), 1.0, atol=0.03)
    assert abs(lag1(Z)) < 0.03


def test_correlated_noise_has_unit_variance_and_the_gaussian_filters_correlation():
    for corr in (2, 8):
        Z = make(seed=corr).noise_field(corr).numpy()
        assert np.allclose(Z.std(axis=(1, 2)), 1.0, atol=1e-12)
        # a Gaussian filter of std s makes the lag-1 correlation exp(-1 / (4 s^2))
        assert abs(lag1(Z) - np.exp(-1.0 / (4 * corr ** 2))) < 0.05
