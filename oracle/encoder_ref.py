"""Oracle for the covariate encoder (Sec. 6, encoder architecture; App.
wildfire experiments, training protocol) and its hybrid gradient.

TEST INFRASTRUCTURE (see oracle/__init__.py): used only by tests, the smoke
check and the benchmark's CPU baseline.

* dense / dense_backward, combine / combine_backward: the definitions of the
  global pathway's dense layer and of G = G0 + alpha G_local,
  b = b0 + alpha b_local, written out in float64 numpy.
* network: the spatial pathway (3x3 convolutions with zero padding, ReLU,
  1x1 heads) and the global pathway, in float64 PyTorch on the CPU, with the
  stored activations rounded to bfloat16 where the kernels store them
  (input, every convolution output); the convolution itself is a library
  step (torch conv2d as the cross-correlation of the definition).
* hybrid_gradient: the parameter gradient of the data term: encoder forward,
  feasibility projection, FP64 solve, implicit adjoint (the oracle's VJP),
  projection VJP, then the encoder's backward by autograd of the forward
  (the gradient is the derivative of the definition; bfloat16 rounding is
  passed through as the identity, as a straight-through estimate).
"""
from __future__ import annotations

import numpy as np

BASE_PLANES = 5  # g11, g12, g22, b1, b2


def dense(x, W, b, relu):
    """y[r][o] = act(b[o] + sum_i W[o][i] x[r][i])."""
    y = np.asarray(x, np.float64) @ np.asarray(W, np.float64).T
    if b is not None:
        y = y + np.asarray(b, np.float64)
    return np.maximum(y, 0.0) if relu else y


def dense_backward(x, W, y, relu, dy):
    """(dx, dW, db) of dense for the upstream gradient dy."""
    g = np.where(np.asarray(y) > 0, dy, 0.0) if relu else np.asarray(dy, np.float64)
    return g @ np.asarray(W, np.float64), g.T @ np.asarray(x, np.float64), g.sum(axis=0)


def combine(base, local, alpha):
    """base (5,), local (5, ...) -> M (3, ...), omega (2, ...)."""
    full = np.asarray(base, np.float64).reshape((BASE_PLANES,) + (1,) * (np.ndim(local) - 1)) + \
        alpha * np.asarray(local, np.float64)
    return full[:3], full[3:]


def combine_backward(dM, dom, alpha):
    """(dlocal, dbase) of combine for upstream gradients dM (3, ...), dom (2, ...)."""
    d = np.concatenate([np.asarray(dM, np.float64), np.asarray(dom, np.float64)])
    return alpha * d, d.reshape(BASE_PLANES, -1).sum(axis=1)


# ---------------------------------------------------------------------------
# the whole encoder in float64 PyTorch (CPU)

def _bf16(t, on):
    """Round to the nearest bfloat16 (ties to even) in the forward pass, the
    identity in the backward pass."""
    import torch
    if not on:
        return t
    r = t.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
    return t + (r - t).detach()


def network(params, X, y, alpha, conv_names, n_heads=BASE_PLANES, bf16=True):
    """params: dict of float64 CPU tensors (requires_grad as the caller wants):
    '<conv>.w' (9, Cout, Cin) with tap t at offset (t // 3 - 1, t % 3 - 1) in
    (y, x), '<conv>.b' (Cout,), 'head<k>.w' (C,), 'head<k>.b' (1,), 'g1.w',
    'g1.b', 'g2.w', 'g2.b' (dense layers of the global pathway, ReLU after
    g1). X (Cin0, H, W) spatial covariates (zero-padded to the first layer's
    Cin), y (Cg,) global covariates. Returns (M (3, H, W), omega (2, H, W))."""
    import torch
    import torch.nn.functional as F
    a = _bf16(X.unsqueeze(0), bf16)
    for name in conv_names:
        w = params[name + ".w"]
        cout, cin = w.shape[1], w.shape[2]
        k = w.reshape(3, 3, cout, cin).permute(2, 3, 0, 1)  # (Cout, Cin, ky, kx)
        a = _bf16(torch.relu(F.conv2d(a, _bf16(k, bf16), params[name + ".b"], padding=1)), bf16)
    local = torch.stack([(a[0] * params[f"head{k}.w"].view(-1, 1, 1)).sum(0) + params[f"head{k}.b"]
                         for k in range(n_heads)])
    h = torch.relu(params["g1.w"] @ y + params["g1.b"])
    base = params["g2.w"] @ h + params["g2.b"]
    full = base.view(-1, 1, 1) + alpha * local
    return full[:3], full[3:]


def hybrid_gradient(params_np, X, y, alpha, conv_names, h, src_idx, src_t, T_obs, mask, bf16=True):
    """Parameter gradients of L = 1/2 sum_{mask} (T - T_obs)^2 through the
    projection and the FP64 solve; returns (dict of numpy gradients, L, M, omega)."""
    import torch

    import oracle
    from synthetic.fields import Problem
    params = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in params_np.items()}
    Xt = torch.tensor(np.asarray(X, np.float64))
    yt = torch.tensor(np.asarray(y, np.float64))
    M, om = network(params, Xt, yt, alpha, conv_names, bf16=bf16)
    Mn, on = M.detach().numpy(), om.detach().numpy()
    Mp, op = oracle.project(Mn, on)
    ny, nx = Mn.shape[1:]
    p = Problem(nx, ny, h, Mp, op, np.asarray(src_idx, np.int32), np.asarray(src_t, np.float64))
    T, _, _ = oracle.forward(p)
    par, _ = oracle.parents_levels(p, T)
    r = np.where(mask, T - T_obs, 0.0)
    L = 0.5 * float(np.sum(r * r))
    dMp, dop, _ = oracle.vjp(p, T, par, r)
    dM, dom = oracle.project_vjp(Mn, on, dMp, dop)
    (M * torch.tensor(dM)).sum().add((om * torch.tensor(dom)).sum()).backward()
    return {k: v.grad.numpy() for k, v in params.items()}, L, Mn, on
