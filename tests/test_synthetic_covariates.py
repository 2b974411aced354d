"""The synthetic covariate scenes are valid Randers data: deterministic per
seed, covariates in [0, 1], an SPD hidden metric, a hidden drift strictly
inside the Randers bound (|b|_{G^-1} <= 0.6 wind speed < 1), an interior
ignition."""
import numpy as np

from synthetic.covariates import scene


def test_scene_is_deterministic_and_valid():
    for seed in (0, 7, 123):
        a, b = scene(seed, n=48), scene(seed, n=48)
        assert np.array_equal(a.X, b.X) and np.array_equal(a.M, b.M) and np.array_equal(a.src_idx, b.src_idx)
        assert a.X.shape == (4, 48, 48) and a.y.shape == (4,)
        assert a.X.min() >= 0.0 and a.X.max() <= 1.0
        m11, m12, m22 = a.M
        assert np.all(m11 > 0) and np.all(m11 * m22 - m12 * m12 > 0)
        det = m11 * m22 - m12 * m12
        bx, by = a.omega
        rho = np.sqrt((bx * bx * m22 - 2 * bx * by * m12 + by * by * m11) / det)
        assert rho.max() <= 0.6 * a.y[2] + 1e-12 and rho.max() < 1.0
        j, i = divmod(int(a.src_idx[0]), 48)
        assert 0 < i < 47 and 0 < j < 47
    assert not np.array_equal(scene(1, n=32).X, scene(2, n=32).X)
