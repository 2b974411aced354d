"""The C-ABI library loads and exports every entry point include/eik.h and
include/eik_inverse.h declare; host-side argument checks reject bad calls before any launch.
No kernel runs here (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    """eik_* functions declared in include/*.h (the solver and the inverse-problem headers)."""
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(eik_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("eik_forward", "eik_backward", "eik_project", "eik_project_backward", "eik_workspace_bytes",
                 "eik_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2603_00035_amd import _lib as L
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(L.EXPORTS) <= set(declared_functions())


def grid(nx=64, ny=64, h=0.1, n_src=1, src=1):
    from paper_2603_00035_amd import _lib as L
    return L.EikGrid(nx, ny, h, n_src, src, None)


def test_workspace_size_and_invalid_grids():
    from paper_2603_00035_amd import _lib as L
    lib = L.lib()
    small = lib.eik_workspace_bytes(ctypes.byref(grid()), L.EIK_F32)
    big = lib.eik_workspace_bytes(ctypes.byref(grid(512, 512)), L.EIK_F32)
    dbl = lib.eik_workspace_bytes(ctypes.byref(grid(512, 512)), L.EIK_F64)
    assert 0 < small < big < dbl
    for bad in (grid(0, 5), grid(5, 5, h=0.0), grid(5, 5, n_src=0), grid(5, 5, src=0)):
        assert lib.eik_workspace_bytes(ctypes.byref(bad), L.EIK_F32) == 0
    assert lib.eik_workspace_bytes(ctypes.byref(grid()), 7) == 0


@pytest.mark.parametrize("case", ["null_fields", "negative_tol", "rounds", "dtype", "workspace"])
def test_forward_rejects_bad_arguments_on_host(case):
    from paper_2603_00035_amd import _lib as L
    lib = L.lib()
    g = grid()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: the checks run before any launch
    args = dict(dtype=L.EIK_F32, M=fake, om=fake, tol=1e-5, rounds=10, ws=fake, wsb=1 << 40)
    if case == "null_fields":
        args["M"] = None
    elif case == "negative_tol":
        args["tol"] = -1.0
    elif case == "rounds":
        args["rounds"] = 0
    elif case == "dtype":
        args["dtype"] = 3
    elif case == "workspace":
        args["wsb"] = 16
    rc = lib.eik_forward(ctypes.byref(g), args["dtype"], args["M"], args["om"], None, args["tol"], args["rounds"],
                         0, fake, fake, fake, args["ws"], args["wsb"], None, None, None)
    assert rc == (-4 if case == "workspace" else -1)
    assert lib.eik_last_error()


def test_project_rejects_bad_parameters():
    from paper_2603_00035_amd import _lib as L
    lib = L.lib()
    fake = ctypes.c_void_p(0x1000)
    p = L.EikProjectParams(1e-3, 1e3, 1e3, 1.5)  # rho_max must be < 1
    assert lib.eik_project(10, L.EIK_F32, fake, fake, fake, fake, ctypes.byref(p), None) == -1
    assert lib.eik_project(0, L.EIK_F32, None, None, None, None, None, None) == 0


@pytest.mark.parametrize("case", ["too_large", "timing", "null_fields"])
def test_noalloc_forward_rejects_on_host(case):
    """The allocation-free forward refuses grids whose workspace exceeds its
    static array, and the timing flag, before touching the device."""
    from paper_2603_00035_amd import _lib as L
    lib = L.lib()
    cap = lib.eik_noalloc_max_workspace_bytes()
    assert cap == 64 << 20
    g = grid(2048, 2048) if case == "too_large" else grid()
    assert case != "too_large" or lib.eik_workspace_bytes(ctypes.byref(g), L.EIK_F32) > cap
    fake = ctypes.c_void_p(0x1000)
    flags = L.EIK_TIME_KERNELS if case == "timing" else 0
    rc = lib.eik_forward_noalloc(ctypes.byref(g), L.EIK_F32, None if case == "null_fields" else fake, fake, None,
                                 1e-5, 10, flags, fake, fake, None, None, None, None)
    assert rc == (L.EIK_EWORKSPACE if case == "too_large" else L.EIK_EINVAL)
    msg = lib.eik_last_error().decode()
    assert msg and (case != "too_large" or "static workspace" in msg)


@pytest.mark.parametrize("case", ["x_stride", "x_offset", "y_offset", "x_pointer", "w_pointer", "y_pointer",
                                  "wgrad_dy_offset", "wgrad_x_pointer"])
def test_network_kernels_reject_unaligned_layouts_on_host(case):
    """The staged convolutions move 8 channels per 16-byte access; layouts that
    would misalign those accesses are refused before any launch."""
    from paper_2603_00035_amd import unet
    lib = unet._bind()
    X, Wt, Y = 0x10000, 0x20000, 0x30000
    if case.startswith("wgrad"):
        args = dict(x=X, x_cs=32, x_co=0, dy=Y, dy_cs=32, dy_co=0)
        if case == "wgrad_dy_offset":
            args.update(dy_cs=48, dy_co=4)
        else:
            args.update(x=X + 8)
        assert lib.eiku_conv_wgrad(0, 1, 8, 8, args["x"], args["x_cs"], args["x_co"], 16, args["dy"], args["dy_cs"],
                                   args["dy_co"], 16, Wt, None) == -1
        return
    args = dict(x=X, x_cs=32, x_co=0, w=Wt, y=Y, y_cs=32, y_co=0)
    args.update({"x_stride": dict(x_cs=36), "x_offset": dict(x_cs=48, x_co=4), "y_offset": dict(y_cs=48, y_co=2),
                 "x_pointer": dict(x=X + 8), "w_pointer": dict(w=Wt + 4), "y_pointer": dict(y=Y + 2)}[case])
    assert lib.eiku_conv_fwd(0, 1, 8, 8, args["x"], args["x_cs"], args["x_co"], 16, args["w"], None, 0, args["y"],
                             args["y_cs"], args["y_co"], 16, None) == -1


@pytest.mark.parametrize("case", ["ca_4", "ca_8", "xb_offset", "xb_slice", "xa_pointer", "xb_pointer",
                                  "wgrad_dy_offset", "wgrad_xb_slice"])
def test_concatenated_input_forms_reject_bad_layouts_on_host(case):
    """The two-source convolution and weight gradient check both sources'
    channel counts, strides, offsets and alignment before any launch."""
    from paper_2603_00035_amd import unet
    lib = unet._bind()
    Xa, Xb, Wt, Y = 0x10000, 0x20000, 0x30000, 0x40000
    a = dict(xa=Xa, xa_cs=16, xa_co=0, Ca=16, xb=Xb, xb_cs=16, xb_co=0, Cb=16)
    a.update({"ca_4": dict(Ca=4, xa_cs=16), "ca_8": dict(Ca=8, xa_cs=8),
              "xb_offset": dict(xb_cs=24, xb_co=4), "xb_slice": dict(xb_cs=16, xb_co=8), "xa_pointer": dict(xa=Xa + 8),
              "xb_pointer": dict(xb=Xb + 8), "wgrad_dy_offset": {}, "wgrad_xb_slice": dict(xb_cs=16, xb_co=8)}[case])
    src = (a["xa"], a["xa_cs"], a["xa_co"], a["Ca"], a["xb"], a["xb_cs"], a["xb_co"], a["Cb"])
    if case.startswith("wgrad"):
        dy_co = 4 if case == "wgrad_dy_offset" else 0
        assert lib.eiku_conv_wgrad_cat(1, 8, 8, *src, Y, 32, dy_co, 16, Wt, None) == -1
        return
    assert lib.eiku_conv_fwd_cat(1, 8, 8, *src, Wt, None, 0, Y, 16, 0, 16, None) == -1


@pytest.mark.parametrize("case", ["tau_zero", "tau_inf", "side", "tol", "cycles", "workspace"])
def test_soft_mode_rejects_bad_arguments_on_host(case):
    """The soft-min entry points check tau, the side limit of one line per
    workgroup, tol, the cycle budget and the workspace before any launch."""
    import ctypes
    from paper_2603_00035_amd import _lib as L
    lib = L.lib()
    nx, ny = (4097, 2) if case == "side" else (16, 16)
    g = L.EikGrid(nx, ny, 0.1, 1, 0x1000, None)
    need = lib.eik_soft_workspace_bytes(ctypes.byref(g), L.EIK_F64)
    assert need >= nx * ny * (28 * 8 + 1)
    tau = {"tau_zero": 0.0, "tau_inf": float("inf")}.get(case, 0.01)
    tol = -1.0 if case == "tol" else 1e-12
    cycles = 0 if case == "cycles" else 8
    ws_bytes = need - 1 if case == "workspace" else need
    M, om, T, ws = 0x10000, 0x20000, 0x30000, 0x40000
    rc = lib.eik_soft_forward(ctypes.byref(g), L.EIK_F64, M, om, tau, tol, cycles, T, ws, ws_bytes, None, None)
    assert rc == (L.EIK_EWORKSPACE if case == "workspace" else L.EIK_EINVAL)
    rc = lib.eik_soft_backward(ctypes.byref(g), L.EIK_F64, M, om, T, tau, 0x50000, tol, cycles, 0x60000, 0x70000,
                               0x80000, ws, ws_bytes, None, None)
    assert rc == (L.EIK_EWORKSPACE if case == "workspace" else L.EIK_EINVAL)
