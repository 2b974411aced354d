"""The learned warm start with the committed weights (trained by the project's
own BF16 MFMA kernels on 20k cold solves of the 256^2 recipe): on held-out
seeds the warm-started solve must reach the cold-start fixed point within 1e-5
(the fixed point does not depend on the initial field), and the comparison of
sweeps and time against the cold start is reported."""
import os

import numpy as np
import pytest

from tests.gpu_common import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_warm_start_reaches_cold_fixed_point_and_reports_gain():
    from paper_2603_00035_amd import warmstart as W
    from paper_2603_00035_amd.unet import UNet
    assert os.path.exists(W.WEIGHTS), "trained weights missing"
    net = UNet()
    net.load_state_dict(torch.load(W.WEIGHTS, weights_only=True))
    seeds = list(range(1_000_000, 1_000_032))
    res = W.evaluate(net, seeds, chunk=32, log=say)
    say(f"[warm] cold {res['cold_s'] * 1e3:.1f} ms, {res['cold_sweeps_per_node']:.1f} sweeps/node; warm "
        f"{res['warm_s'] * 1e3:.1f} ms (incl. inference {res['infer_s'] * 1e3:.1f} ms), "
        f"{res['warm_sweeps_per_node']:.1f} sweeps/node; with fallback {res['warm_fb_s'] * 1e3:.1f} ms; "
        f"prediction mean rel err {np.mean(res['pred_rel_err_mean']):.2e}")
    assert res["max_rel_warm_vs_cold"] <= 1e-5
    assert np.mean(res["pred_rel_err_mean"]) < 0.2  # the network predicts T, not noise
