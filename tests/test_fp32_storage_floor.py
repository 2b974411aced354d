"""How far from the exact gradient a solve that stores T in single precision
can get, measured on the oracle alone (CPU).

The adjoint's donor weights w = mu1 / (mu1 + mu2) of a two-point update
(Sec. 3.3, Eq. jacobian_planar) are functions of the donor-time difference
divided by the grid spacing, so a relative error e in the stored times moves
them by about e * T / h: on a 512 x 512 grid single-precision rounding alone
(e ~ 6e-8) reaches the 1e-4 gradient bar. The oracle's Gauss-Seidel sweeps
with every stored value rounded to single precision (each update still exact
in double) give the best field such a solve can hold; its gradient of the
512 x 512 workload's 256-cell loss is compared here with the exact one. The
GPU tests hold single-precision runs against this measured floor and the
mixed-precision path, which stores T in double after the single-precision
sweeps, against 1e-4.
"""
import numpy as np
import pytest

import oracle
from synthetic.fields import Problem, make_problem


def rel_l2(a, b):
    a = np.concatenate([x.ravel() for x in a])
    b = np.concatenate([x.ravel() for x in b])
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def loss_grad(T, cells, target):
    g = np.zeros_like(T)
    g.flat[cells] = 2.0 * (T.flat[cells] - target.flat[cells]) / len(cells)
    return g


@pytest.fixture(scope="module")
def c2():
    p = make_problem("c2", 0)
    q = p.rounded(np.float32)
    To, _, st = oracle.forward(q)
    assert st == 0
    T32, _, st32 = oracle.forward(q, mode="gs_f32")
    assert st32 == 0
    tgt = make_problem("c2", 1).rounded(np.float32)
    Tt, _, _ = oracle.forward(Problem(q.nx, q.ny, q.h, tgt.M, tgt.omega, q.src_idx, q.src_t))
    return p, q, To, T32, Tt


def test_fp32_storage_keeps_the_field_but_not_the_gradient(c2):
    p, q, To, T32, Tt = c2
    # every stored value is a single-precision number and the field is a
    # fixed point of the rounded update
    assert np.array_equal(T32, T32.astype(np.float32).astype(np.float64))
    v, _ = oracle.local_update_all(q, T32)
    m = np.isfinite(To)
    m.flat[p.src_idx] = False
    assert np.array_equal(v[m].astype(np.float32).astype(np.float64), T32[m])
    # the forward bar holds with a wide margin
    fwd = float(np.max(np.abs(T32[m] - To[m]) / To[m]))
    assert fwd < 1e-6
    po, _ = oracle.parents_levels(q, To)
    p32, _ = oracle.parents_levels(q, T32)
    dMo, domo, dso = oracle.vjp(q, To, po, loss_grad(To, p.loss_idx, Tt))
    dM3, dom3, ds3 = oracle.vjp(q, T32, p32, loss_grad(T32, p.loss_idx, Tt))
    floor = rel_l2([dM3, dom3], [dMo, domo])
    print(f"single-precision storage: forward {fwd:.2e}, parameter gradient {floor:.3e}")
    # the parameter gradient sits at the 1e-4 bar (1.005e-4 on this workload):
    # no single-precision field can be relied on to meet it
    assert 8e-5 < floor < 2e-4
    # with the source-time gradients in the norm the same fields agree to
    # ~6e-7: those entries carry the loss's total mass (the donor weights sum
    # to one) and dominate the norm, so they hide the parameter error
    assert rel_l2([dM3, dom3, ds3], [dMo, domo, dso]) < 5e-6
    # the same stencils on both fields: the difference is in the weights
    dM4, dom4, _ = oracle.vjp(q, T32, po, loss_grad(T32, p.loss_idx, Tt))
    assert rel_l2([dM4, dom4], [dMo, domo]) == pytest.approx(floor, rel=0.05)


def test_gradient_sensitivity_to_field_noise(c2):
    """Random relative perturbations s of the exact field move the parameter
    gradient in proportion to s (about 500 s here): the weights are difference
    quotients of T at the grid scale."""
    p, q, To, _, Tt = c2
    po, _ = oracle.parents_levels(q, To)
    dMo, domo, _ = oracle.vjp(q, To, po, loss_grad(To, p.loss_idx, Tt))
    rng = np.random.default_rng(0)
    r = []
    for s in (1e-8, 1e-7):
        Tp = To * (1.0 + s * rng.standard_normal(To.shape))
        Tp.flat[p.src_idx] = To.flat[p.src_idx]
        dM, dom, _ = oracle.vjp(q, Tp, po, loss_grad(Tp, p.loss_idx, Tt))
        r.append(rel_l2([dM, dom], [dMo, domo]))
    assert 2e-6 < r[0] < 2e-5 and 2e-5 < r[1] < 2e-4
    assert 5 < r[1] / r[0] < 20
