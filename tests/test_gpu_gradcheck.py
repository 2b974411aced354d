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


@pytest.mark.parametrize("name", ["isotropic", "anisotropic", "drift"])
def test_gpu_gradient_against_oracle_finite_differences(name):
    """The GPU's implicit gradient at 20 random interior entries against
    central differences (eps = 1e-5) of the oracle's own FP64 solve, each
    entry kept only where the oracle's active stencils at +-eps equal the
    unperturbed ones: the check is independent of the GPU's forward."""
    import numpy as np

    import oracle
    from paper_2603_00035_amd import gradcheck as C
    from synthetic.fields import Problem
    chk = C.Check(name, n=64, seed=3)
    n, eps = chk.n, 1e-5
    M, om = chk.M.cpu().numpy(), chk.om.cpu().numpy()
    src = chk.src.cpu().numpy()
    c = chk.c.cpu().numpy()
    base = Problem(n, n, chk.h, M, om, src, np.zeros(1))
    T0, _, st = oracle.forward(base)
    assert st == 0
    par0, _ = oracle.parents_levels(base, T0)
    dM, dom = chk.grad(chk.M, chk.om)
    dM, dom = dM.cpu().numpy(), dom.cpu().numpy()
    rng = np.random.default_rng(5)
    planes = C.PLANES[name]
    errs, skipped = [], 0
    while len(errs) < 20:
        which = planes[rng.integers(len(planes))]
        arr, g = (M, dM) if which == "M" else (om, dom)
        comp = int(rng.integers(arr.shape[0]))
        j, i = (int(x) for x in rng.integers(2, n - 2, 2))
        an = float(g[comp, j, i])
        if abs(an) < 1e-8 * float(np.abs(g).max()):
            continue
        sides = []
        for s in (eps, -eps):
            P = arr.copy()
            P[comp, j, i] += s
            prob = Problem(n, n, chk.h, P if which == "M" else M, om if which == "M" else P, src, np.zeros(1))
            T, _, st = oracle.forward(prob, T_init=T0)
            assert st == 0
            par, _ = oracle.parents_levels(prob, T)
            sides.append((T, par))
        if not all(np.array_equal(p, par0) for _, p in sides):
            skipped += 1
            continue
        fd = float(np.sum(c * (sides[0][0] - sides[1][0]))) / (2 * eps)
        errs.append(abs(fd - an) / abs(an))
    say(f"[gradcheck vs oracle FD] {name}: max rel error {max(errs):.2e} over {len(errs)} entries "
        f"({skipped} skipped at stencil switches)")
    assert max(errs) < 1e-6
