"""The paper's gradient checks on the GPU's FP64 path (Sec. 4, gradient
validation): implicit gradients against central finite differences of the
solver's own output at random interior nodes where the active stencils stay
fixed under the perturbation; random-direction and noise-stability figures
are reported."""
import pytest

from tests.gpu_common import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name", ["isotropic", "anisotropic", "drift"])
def test_pointwise_finite_differences(name):
    from paper_2603_00035_amd import gradcheck as C
    chk = C.Check(name, n=64, seed=1)
    err, tested, skipped = chk.pointwise(points=20, planes=C.PLANES[name])
    say(f"[gradcheck] {name}: max rel error {err:.2e} over {tested} points ({skipped} skipped at stencil switches)")
    assert tested == 20
    assert err < 1e-6


def test_random_directions_and_stability_are_reported():
    from paper_2603_00035_amd import gradcheck as C
    chk = C.Check("anisotropic", n=64, seed=2)
    f10, f1, med = chk.random_directions(count=20)
    stab = chk.stability(trials=4)
    say(f"[gradcheck] random directions: {f10:.2f} within 10 %, {f1:.2f} within 1 %, median error {med:.2e}; "
        f"1 % metric noise: field {100 * stab['field_rel_l2']:.2f} %, interior entries mean "
        f"{100 * stab['interior_mean']:.2f} % median {100 * stab['interior_median']:.2f} %")
    # directions of unit length move each parameter by ~eps / sqrt(3 n^2), so
    # few active stencils switch and the directional derivatives agree
    assert f10 >= 0.9
    assert stab["field_rel_l2"] < 0.5
