"""Pins of the covariate encoder's oracle (oracle/encoder_ref.py) against
facts other than its own formulas: a worked example, special cases, central
differences, the shift a single convolution tap makes, and central
differences of the whole hybrid loss through the FP64 solve."""
import numpy as np
import pytest

from oracle import encoder_ref as R

torch = pytest.importorskip("torch")


def test_dense_worked_example():
    # x = (1, -2), W = [[1, 2], [3, 4]], b = (0.5, -1):
    # W x + b = (1 - 4 + 0.5, 3 - 8 - 1) = (-2.5, -6); a third output (0, 1) . x + 4 = 2
    x = np.array([[1.0, -2.0]])
    W = np.array([[1.0, 2.0], [3.0, 4.0], [0.0, 1.0]])
    b = np.array([0.5, -1.0, 4.0])
    assert np.array_equal(R.dense(x, W, b, False), [[-2.5, -6.0, 2.0]])
    assert np.array_equal(R.dense(x, W, b, True), [[0.0, 0.0, 2.0]])
    # identity weights without bias: the layer is ReLU itself
    z = np.array([[0.3, -0.7, 2.0]])
    assert np.array_equal(R.dense(z, np.eye(3), None, True), [[0.3, 0.0, 2.0]])


@pytest.mark.parametrize("relu", [False, True])
def test_dense_backward_matches_central_differences(relu):
    rng = np.random.default_rng(3)
    x, W, b = rng.normal(size=(3, 5)), rng.normal(size=(4, 5)), rng.normal(size=4)
    dy = rng.normal(size=(3, 4))
    y = R.dense(x, W, b, relu)
    dx, dW, db = R.dense_backward(x, W, y, relu, dy)
    f = lambda x_, W_, b_: float(np.sum(dy * R.dense(x_, W_, b_, relu)))
    eps = 1e-6
    for arr, got, which in ((x, dx, 0), (W, dW, 1), (b, db, 2)):
        for idx in np.ndindex(arr.shape):
            P, Q = [x.copy(), W.copy(), b.copy()], [x.copy(), W.copy(), b.copy()]
            P[which][idx] += eps
            Q[which][idx] -= eps
            fd = (f(*P) - f(*Q)) / (2 * eps)
            assert abs(fd - got[idx]) <= 1e-6 * (1 + abs(fd))


def test_combine_special_cases_and_backward():
    rng = np.random.default_rng(4)
    base = rng.normal(size=5)
    local = rng.normal(size=(5, 3, 4))
    M, om = R.combine(base, local, 0.0)
    assert np.array_equal(M, np.broadcast_to(base[:3, None, None], (3, 3, 4)))
    assert np.array_equal(om, np.broadcast_to(base[3:, None, None], (2, 3, 4)))
    M, om = R.combine(np.zeros(5), local, 1.0)
    assert np.array_equal(np.concatenate([M, om]), local)
    dM, dom = rng.normal(size=(3, 3, 4)), rng.normal(size=(2, 3, 4))
    dl, dbase = R.combine_backward(dM, dom, 0.7)
    f = lambda bs, lc: float(np.sum(dM * R.combine(bs, lc, 0.7)[0]) + np.sum(dom * R.combine(bs, lc, 0.7)[1]))
    eps = 1e-6
    for c in range(5):
        e = np.zeros(5)
        e[c] = eps
        assert abs((f(base + e, local) - f(base - e, local)) / (2 * eps) - dbase[c]) < 1e-7
    E = np.zeros_like(local)
    E[2, 1, 3] = eps
    assert abs((f(base, local + E) - f(base, local - E)) / (2 * eps) - dl[2, 1, 3]) < 1e-7


def small_params(rng, names=("a", "b"), cin=16, hid=4, n_cov=3, n_global=4, hidden=5):
    p = {}
    c = cin
    for nm in names:
        p[nm + ".w"] = rng.normal(size=(9, hid, c)) * 0.4
        p[nm + ".b"] = rng.normal(size=hid) * 0.1
        c = hid
    p["a.w"][:, :, n_cov:] = 0.0
    for k in range(5):
        p[f"head{k}.w"] = rng.normal(size=hid) * 0.05
        p[f"head{k}.b"] = np.zeros(1)
    p["g1.w"] = rng.normal(size=(hidden, n_global))
    p["g1.b"] = rng.normal(size=hidden) * 0.1
    p["g2.w"] = rng.normal(size=(5, hidden)) * 0.02
    p["g2.b"] = np.array([1.0, 0.0, 1.0, 0.0, 0.0])
    return p


def test_single_tap_shifts_the_input():
    """A convolution whose only weight is tap t = 3 (ky + 1) + (kx + 1)
    copies x(y + ky, x + kx): the tap layout of the definition."""
    rng = np.random.default_rng(6)
    X = rng.uniform(0.5, 1.0, size=(16, 7, 8))
    X[1:] = 0.0
    for t in range(9):
        p = small_params(rng, names=("a",), hid=1, n_cov=1)
        p["a.w"][:] = 0.0
        p["a.w"][t, 0, 0] = 1.0
        p["a.b"][:] = 0.0
        p["head0.w"][:] = 1.0
        p["head0.b"][:] = 0.0
        P = {k: torch.tensor(v) for k, v in p.items()}
        M, _ = R.network(P, torch.tensor(X), torch.zeros(4, dtype=torch.float64), 1.0, ["a"], bf16=False)
        out = M[0].numpy() - float(P["g2.b"][0] + P["g2.w"][0] @ torch.relu(P["g1.b"]))
        ky, kx = t // 3 - 1, t % 3 - 1
        ref = np.zeros((7, 8))
        for yy in range(7):
            for xx in range(8):
                if 0 <= yy + ky < 7 and 0 <= xx + kx < 8:
                    ref[yy, xx] = X[0, yy + ky, xx + kx]
        assert np.allclose(out, ref, atol=1e-12)


def test_hybrid_gradient_matches_central_differences():
    """The whole chain (network, projection, FP64 solve, data term) against
    central differences of the loss, without bfloat16 rounding."""
    from synthetic.covariates import scene
    import oracle
    from synthetic.fields import Problem
    sc = scene(11, n=12)
    rng = np.random.default_rng(7)
    p = small_params(rng, n_cov=4)
    X = np.zeros((16, 12, 12))
    X[:4] = sc.X
    Tt, _, _ = oracle.forward(Problem(12, 12, sc.h, sc.M, sc.omega, sc.src_idx, np.zeros(1)))
    mask = rng.uniform(size=(12, 12)) < 0.6
    g, L0, _, _ = R.hybrid_gradient(p, X, sc.y, 0.5, ["a", "b"], sc.h, sc.src_idx, np.zeros(1), Tt, mask,
                                    bf16=False)

    def loss(q):
        P = {k: torch.tensor(v) for k, v in q.items()}
        M, om = R.network(P, torch.tensor(X), torch.tensor(sc.y), 0.5, ["a", "b"], bf16=False)
        Mp, op = oracle.project(M.numpy(), om.numpy())
        T, _, _ = oracle.forward(Problem(12, 12, sc.h, Mp, op, sc.src_idx, np.zeros(1)))
        r = np.where(mask, T - Tt, 0.0)
        return 0.5 * float(np.sum(r * r))

    assert abs(loss(p) - L0) <= 1e-12 * abs(L0)
    eps = 1e-6
    checked = 0
    for key, idx in (("g2.b", (0,)), ("g2.b", (4,)), ("g1.w", (1, 2)), ("head1.w", (2,)), ("b.w", (4, 1, 3)),
                     ("a.b", (2,))):
        P, Q = {k: v.copy() for k, v in p.items()}, {k: v.copy() for k, v in p.items()}
        P[key][idx] += eps
        Q[key][idx] -= eps
        fd = (loss(P) - loss(Q)) / (2 * eps)
        assert abs(fd - g[key][idx]) <= 1e-5 * max(abs(fd), 1e-3 * abs(L0)), (key, idx, fd, g[key][idx])
        checked += 1
    assert checked == 6
