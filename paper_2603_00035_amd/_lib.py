"""ctypes binding of ``libeik.so`` (the C ABI in include/eik.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. Loading fails loudly when the library has not been built; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads PyTorch's HIP runtime first; the library then binds to the same one

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeik.so")

EIK_F32, EIK_F64 = 0, 1
EIK_OK, EIK_NOT_CONVERGED = 0, 1
EIK_EINVAL, EIK_EINFEASIBLE, EIK_EDEVICE, EIK_EWORKSPACE = -1, -2, -3, -4
EIK_SCHED_ROUNDS, EIK_SCHED_QUEUE = 1, 2
EIK_CHECK_FEASIBLE = 1
EIK_TIME_KERNELS = 2
EIK_WARM_FALLBACK = 4
EIK_MIXED = 2  # dtype code of the batched mixed-precision workspace, plan and pending calls
STATUS_NAMES = {0: "EIK_OK", 1: "EIK_NOT_CONVERGED", -1: "EIK_EINVAL", -2: "EIK_EINFEASIBLE",
                -3: "EIK_EDEVICE", -4: "EIK_EWORKSPACE"}
SOURCE, UNREACHED = 0xFE, 0xFF

EXPORTS = ["eik_workspace_bytes", "eik_forward", "eik_backward", "eik_project", "eik_project_backward",
           "eik_last_error", "eik_batch_workspace_bytes", "eik_batch_plan", "eik_forward_batched",
           "eik_backward_batched", "eik_batch_pending", "eik_mixed_workspace_bytes", "eik_forward_mixed",
           "eik_backward_mixed", "eik_inv_scratch_bytes", "eik_tv", "eik_obs_loss", "eik_sum_sq", "eik_param_step",
           "eik_tie_isotropic", "eik_enc_dense", "eik_enc_dense_backward", "eik_enc_combine",
           "eik_enc_scratch_bytes", "eik_enc_combine_backward", "eik_forward_noalloc",
           "eik_noalloc_max_workspace_bytes", "eik_tv_log_euclid", "eik_tv_log_euclid_work_bytes",
           "eik_forward_batched_mixed", "eik_backward_batched_mixed", "eik_soft_workspace_bytes",
           "eik_soft_forward", "eik_soft_backward", "eik_soft_batch_workspace_bytes", "eik_soft_forward_batched",
           "eik_soft_backward_batched"]


class EikGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("h", ctypes.c_double),
                ("n_src", ctypes.c_int32), ("src_idx", ctypes.c_void_p), ("src_t", ctypes.c_void_p)]


class EikStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("converged", ctypes.c_int32), ("cell_updates", ctypes.c_int64),
                ("n_levels", ctypes.c_int32), ("status", ctypes.c_int32), ("sweep_launches", ctypes.c_int32),
                ("aux_rounds", ctypes.c_int32), ("sweep_ms", ctypes.c_double), ("fast_ms", ctypes.c_double),
                ("fast_cell_updates", ctypes.c_int64), ("fast_launches", ctypes.c_int32), ("fell_back", ctypes.c_int32)]


class EikTuning(ctypes.Structure):
    _fields_ = [("tile_height", ctypes.c_int32), ("max_local_cycles", ctypes.c_int32),
                ("rounds_per_check", ctypes.c_int32), ("fast_cold_start", ctypes.c_int32),
                ("adjoint_rounds", ctypes.c_int32), ("level_rounds", ctypes.c_int32),
                ("scheduler", ctypes.c_int32), ("node_lanes", ctypes.c_int32),
                ("adjoint_cycles", ctypes.c_int32), ("adjoint_waves", ctypes.c_int32),
                ("full_waves", ctypes.c_int32), ("adjoint_mode", ctypes.c_int32), ("level_mode", ctypes.c_int32)]


class EikProjectParams(ctypes.Structure):
    _fields_ = [("eig_min", ctypes.c_double), ("eig_max", ctypes.c_double), ("eucl_clip", ctypes.c_double),
                ("rho_max", ctypes.c_double)]


class EikError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_00035_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        gp = ctypes.POINTER(EikGrid)
        L.eik_workspace_bytes.argtypes = [gp, i32]
        L.eik_workspace_bytes.restype = ctypes.c_size_t
        L.eik_forward.argtypes = [gp, i32, vp, vp, vp, d, i32, i32, vp, vp, vp, vp, ctypes.c_size_t,
                                  ctypes.POINTER(EikTuning), ctypes.POINTER(EikStats), vp]
        L.eik_forward.restype = ctypes.c_int
        L.eik_backward.argtypes = [gp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t,
                                   ctypes.POINTER(EikTuning), ctypes.POINTER(EikStats), vp]
        L.eik_backward.restype = ctypes.c_int
        L.eik_project.argtypes = [i64, i32, vp, vp, vp, vp, ctypes.POINTER(EikProjectParams), vp]
        L.eik_project.restype = ctypes.c_int
        L.eik_project_backward.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(EikProjectParams), vp]
        L.eik_project_backward.restype = ctypes.c_int
        tp = ctypes.POINTER(EikTuning)
        sp = ctypes.POINTER(EikStats)
        L.eik_batch_workspace_bytes.argtypes = [i32, gp, i32]
        L.eik_batch_workspace_bytes.restype = ctypes.c_size_t
        L.eik_batch_plan.argtypes = [i32, gp, i32, tp, vp, ctypes.c_size_t, vp]
        L.eik_batch_plan.restype = ctypes.c_int
        L.eik_forward_batched.argtypes = [i32, gp, i32, vp, vp, vp, vp, vp, d, i32, i32, vp, vp, vp, vp,
                                          ctypes.c_size_t, tp, sp, vp]
        L.eik_forward_batched.restype = ctypes.c_int
        L.eik_backward_batched.argtypes = [i32, gp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                           ctypes.c_size_t, tp, sp, vp]
        L.eik_backward_batched.restype = ctypes.c_int
        L.eik_forward_batched_mixed.argtypes = [i32, gp, vp, vp, vp, vp, d, d, i32, i32, vp, vp, vp, vp,
                                                ctypes.c_size_t, tp, tp, sp, vp]
        L.eik_forward_batched_mixed.restype = ctypes.c_int
        L.eik_backward_batched_mixed.argtypes = [i32, gp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                                 ctypes.c_size_t, tp, sp, vp]
        L.eik_backward_batched_mixed.restype = ctypes.c_int
        L.eik_batch_pending.argtypes = [i32, gp, i32, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int64), vp]
        L.eik_batch_pending.restype = ctypes.c_int
        L.eik_mixed_workspace_bytes.argtypes = [gp]
        L.eik_mixed_workspace_bytes.restype = ctypes.c_size_t
        L.eik_forward_mixed.argtypes = [gp, vp, vp, d, d, i32, i32, vp, vp, vp, vp, ctypes.c_size_t, tp, tp, sp, vp]
        L.eik_forward_mixed.restype = ctypes.c_int
        L.eik_forward_noalloc.argtypes = [gp, i32, vp, vp, vp, d, i32, i32, vp, vp, vp, tp, sp, vp]
        L.eik_forward_noalloc.restype = ctypes.c_int
        L.eik_noalloc_max_workspace_bytes.argtypes = []
        L.eik_noalloc_max_workspace_bytes.restype = ctypes.c_size_t
        L.eik_backward_mixed.argtypes = [gp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, tp, sp, vp]
        L.eik_backward_mixed.restype = ctypes.c_int
        L.eik_inv_scratch_bytes.argtypes = []
        L.eik_inv_scratch_bytes.restype = ctypes.c_size_t
        L.eik_tv.argtypes = [i32, i32, i32, i32, vp, ctypes.POINTER(ctypes.c_double), d, vp, vp, vp, vp]
        L.eik_tv.restype = ctypes.c_int
        L.eik_tv_log_euclid_work_bytes.argtypes = [i32, i32, i32]
        L.eik_tv_log_euclid_work_bytes.restype = ctypes.c_size_t
        L.eik_tv_log_euclid.argtypes = [i32, i32, i32, vp, d, vp, vp, vp, vp, vp]
        L.eik_tv_log_euclid.restype = ctypes.c_int
        L.eik_obs_loss.argtypes = [i64, i32, vp, vp, vp, vp, vp, vp, vp]
        L.eik_obs_loss.restype = ctypes.c_int
        L.eik_sum_sq.argtypes = [i64, i32, vp, vp, vp, vp]
        L.eik_sum_sq.restype = ctypes.c_int
        L.eik_param_step.argtypes = [i64, i32, i32, vp, vp, vp, vp, d, d, d, d, i32, d, vp, vp]
        L.eik_param_step.restype = ctypes.c_int
        L.eik_tie_isotropic.argtypes = [i64, i32, vp, vp]
        L.eik_tie_isotropic.restype = ctypes.c_int
        L.eik_enc_dense.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp, vp]
        L.eik_enc_dense.restype = ctypes.c_int
        L.eik_enc_dense_backward.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp]
        L.eik_enc_dense_backward.restype = ctypes.c_int
        L.eik_enc_combine.argtypes = [i32, i64, i32, d, vp, vp, vp, vp, vp]
        L.eik_enc_combine.restype = ctypes.c_int
        L.eik_enc_scratch_bytes.argtypes = [i32]
        L.eik_enc_scratch_bytes.restype = ctypes.c_size_t
        L.eik_enc_combine_backward.argtypes = [i32, i64, i32, d, vp, vp, vp, vp, vp, vp]
        L.eik_enc_combine_backward.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int32)
        L.eik_soft_workspace_bytes.argtypes = [gp, i32]
        L.eik_soft_workspace_bytes.restype = ctypes.c_size_t
        L.eik_soft_forward.argtypes = [gp, i32, vp, vp, d, d, i32, vp, vp, ctypes.c_size_t, ip, vp]
        L.eik_soft_forward.restype = ctypes.c_int
        L.eik_soft_backward.argtypes = [gp, i32, vp, vp, vp, d, vp, d, i32, vp, vp, vp, vp, ctypes.c_size_t, ip, vp]
        L.eik_soft_backward.restype = ctypes.c_int
        L.eik_soft_batch_workspace_bytes.argtypes = [i32, gp, i32]
        L.eik_soft_batch_workspace_bytes.restype = ctypes.c_size_t
        dpp = ctypes.POINTER(ctypes.c_double)
        L.eik_soft_forward_batched.argtypes = [i32, gp, i32, vp, vp, vp, vp, d, d, i32, vp, vp, ctypes.c_size_t, ip,
                                               dpp, vp]
        L.eik_soft_forward_batched.restype = ctypes.c_int
        L.eik_soft_backward_batched.argtypes = [i32, gp, i32, vp, vp, vp, vp, d, vp, d, i32, vp, vp, vp, vp,
                                                ctypes.c_size_t, ip, dpp, vp]
        L.eik_soft_backward_batched.restype = ctypes.c_int
        L.eik_last_error.argtypes = []
        L.eik_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(fn, code, ok=(EIK_OK,)):
    if code not in ok:
        raise EikError(fn, code, lib().eik_last_error().decode())
    return code


def dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return EIK_F32
    if t.dtype == torch.float64:
        return EIK_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)
