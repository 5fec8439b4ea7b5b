"""ctypes front end of libpsdproj.so (the C ABI in include/psdproj.h).

Argument marshalling only: every step of the projection runs in the HIP
kernels behind the ABI.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsdproj.so")

PSD_OK = 0
STATUS_NAMES = {0: "PSD_OK", 1: "PSD_EINVAL", 2: "PSD_EWORKSPACE", 3: "PSD_ENOMEM",
                4: "PSD_ENONFINITE", 5: "PSD_ENOCONV", 6: "PSD_EDEVICE", 7: "PSD_EUNSUPPORTED"}
MODES = {"fp64": 0, "mixed_bf16": 1, "mixed_fp32": 2, "mixed_bf16x3": 3}
PSD_FLAG_SAVE = 1
PSD_FLAG_WARM = 2
NOALLOC_SCRATCH_BYTES = 48 << 20   # PSD_NOALLOC_SCRATCH_BYTES

# Every symbol include/psdproj.h declares.
EXPORTS = ("psd_workspace_size", "psd_saved_size", "psd_project", "psd_project_warm", "psd_project_noalloc",
           "psd_project_batched",
           "psd_project_vjp", "psd_plan_create", "psd_plan_workspace_size", "psd_plan_concurrency",
           "psd_plan_group_size", "psd_plan_ns_tile_threshold",
           "psd_plan_execute", "psd_plan_tune", "psd_plan_destroy", "psd_timing_start", "psd_timing_stop",
           "psd_set_ns_iterations", "psd_set_mixed_fallback", "psd_status_string", "psd_version",
           "psd_affine_dims", "psd_affine_workspace_size", "psd_constraint_apply", "psd_constraint_adjoint",
           "psd_affine_step", "psd_scs_workspace_size", "psd_scs_solve", "psd_scs_workspace_size_batched",
           "psd_scs_solve_batched")
KF_HEMV, KF_GEMM, KF_NS, KF_WSTEP = 1, 2, 3, 4


class PsdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} ({status_string(status)})")


class PsdInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_pos", ctypes.c_int32), ("n_neg", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("fallback", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("est_rel_err", ctypes.c_double), ("scale", ctypes.c_double)]


class ScsSettings(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("mixed_iters", ctypes.c_int32), ("mixed_mode", ctypes.c_int32), ("normalize", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("anderson", ctypes.c_int32), ("eps", ctypes.c_double),
                ("alpha", ctypes.c_double), ("mixed_switch", ctypes.c_double), ("warm_proj", ctypes.c_int32)]


class ScsInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("proj_status", ctypes.c_int32),
                ("aa_accepted", ctypes.c_int32), ("aa_rejected", ctypes.c_int32),
                ("switch_iter", ctypes.c_int32), ("pobj", ctypes.c_double), ("dobj", ctypes.c_double),
                ("res_pri", ctypes.c_double), ("res_dual", ctypes.c_double), ("gap", ctypes.c_double),
                ("tau", ctypes.c_double), ("kappa", ctypes.c_double), ("sigma", ctypes.c_double),
                ("post_lambda", ctypes.c_double), ("post_lambda_min", ctypes.c_double),
                ("warm_refined", ctypes.c_int32), ("warm_fallbacks", ctypes.c_int32)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_20519_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    L.psd_workspace_size.argtypes = [i32, ctypes.POINTER(i32), i32, i32, ctypes.POINTER(sz)]
    L.psd_workspace_size.restype = i32
    L.psd_saved_size.argtypes = [i32]
    L.psd_saved_size.restype = sz
    L.psd_project.argtypes = [i32, vp, vp, i32, vp, sz, vp, vp, vp]
    L.psd_project.restype = i32
    L.psd_project_warm.argtypes = [i32, vp, vp, vp, vp, vp, sz, vp, vp]
    L.psd_project_warm.restype = i32
    L.psd_project_noalloc.argtypes = [i32, vp, vp, i32, vp, vp]
    L.psd_project_noalloc.restype = i32
    L.psd_project_batched.argtypes = [i32, ctypes.POINTER(i32), vp, vp, i32, vp, sz, vp, vp]
    L.psd_project_batched.restype = i32
    L.psd_project_vjp.argtypes = [i32, vp, vp, vp, vp, i32, vp, sz, vp]
    L.psd_project_vjp.restype = i32
    L.psd_status_string.argtypes = [i32]
    L.psd_status_string.restype = ctypes.c_char_p
    L.psd_version.restype = ctypes.c_char_p
    L.psd_plan_create.argtypes = [i32, ctypes.POINTER(i32), i32, i32, ctypes.POINTER(vp)]
    L.psd_plan_create.restype = i32
    L.psd_plan_workspace_size.argtypes = [vp, i32, ctypes.POINTER(sz)]
    L.psd_plan_workspace_size.restype = i32
    L.psd_plan_concurrency.argtypes = [vp]
    L.psd_plan_concurrency.restype = i32
    L.psd_plan_group_size.argtypes = [vp]
    L.psd_plan_group_size.restype = i32
    L.psd_plan_ns_tile_threshold.argtypes = [vp]
    L.psd_plan_ns_tile_threshold.restype = i32
    L.psd_plan_execute.argtypes = [vp, vp, vp, vp, sz, vp, vp]
    L.psd_plan_execute.restype = i32
    L.psd_plan_tune.argtypes = [vp, vp, vp, vp, sz, vp, i32, ctypes.POINTER(i32)]
    L.psd_plan_tune.restype = i32
    L.psd_plan_destroy.argtypes = [vp]
    L.psd_plan_destroy.restype = i32
    L.psd_set_ns_iterations.argtypes = [i32, i32]
    L.psd_set_ns_iterations.restype = i32
    L.psd_set_mixed_fallback.argtypes = [ctypes.c_double]
    L.psd_set_mixed_fallback.restype = i32
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.psd_affine_dims.argtypes = [i32, i64p, i64p]
    L.psd_affine_dims.restype = i32
    L.psd_affine_workspace_size.argtypes = [i32, ctypes.POINTER(sz)]
    L.psd_affine_workspace_size.restype = i32
    L.psd_constraint_apply.argtypes = [i32, vp, vp, vp, sz, vp]
    L.psd_constraint_apply.restype = i32
    L.psd_constraint_adjoint.argtypes = [i32, vp, vp, vp, sz, vp]
    L.psd_constraint_adjoint.restype = i32
    L.psd_affine_step.argtypes = [i32, vp, vp, vp, vp, vp, sz, vp]
    L.psd_affine_step.restype = i32
    L.psd_scs_workspace_size.argtypes = [ctypes.POINTER(ScsSettings), ctypes.POINTER(sz)]
    L.psd_scs_workspace_size.restype = i32
    L.psd_scs_solve.argtypes = [ctypes.POINTER(ScsSettings), vp, vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(ScsInfo)]
    L.psd_scs_solve.restype = i32
    L.psd_scs_workspace_size_batched.argtypes = [ctypes.POINTER(ScsSettings), i32, ctypes.POINTER(sz)]
    L.psd_scs_workspace_size_batched.restype = i32
    L.psd_scs_solve_batched.argtypes = [ctypes.POINTER(ScsSettings), i32, vp, vp, vp, vp, vp, vp, sz, vp,
                                        ctypes.POINTER(ScsInfo)]
    L.psd_scs_solve_batched.restype = i32
    L.psd_timing_start.argtypes = [i32, i32]
    L.psd_timing_start.restype = i32
    L.psd_timing_stop.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.psd_timing_stop.restype = i32
    _lib = L
    return L


def status_string(st: int) -> str:
    try:
        return lib().psd_status_string(st).decode()
    except RuntimeError:
        return STATUS_NAMES.get(st, "?")


def check(st: int, what: str):
    if st != PSD_OK:
        raise PsdError(st, what)


def int_array(vals):
    arr = (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])
    return arr


def workspace_size(sizes, mode: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    arr = int_array(sizes)
    check(lib().psd_workspace_size(len(sizes), arr, mode, flags, ctypes.byref(out)), "psd_workspace_size")
    return int(out.value)


def saved_size(n: int) -> int:
    return int(lib().psd_saved_size(n))


def timing_start(family: int, max_launches: int):
    check(lib().psd_timing_start(family, max_launches), "psd_timing_start")


def timing_stop():
    """-> (total ms, launches timed, algorithmic work)"""
    ms, n, wk = ctypes.c_double(0), ctypes.c_int32(0), ctypes.c_double(0)
    check(lib().psd_timing_stop(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(wk)), "psd_timing_stop")
    return ms.value, n.value, wk.value


def set_ns_iterations(iters: int, corrections: int):
    check(lib().psd_set_ns_iterations(iters, corrections), "psd_set_ns_iterations")


def set_mixed_fallback(max_rel_err: float):
    check(lib().psd_set_mixed_fallback(float(max_rel_err)), "psd_set_mixed_fallback")


def affine_dims(d: int):
    """(nx, ny): lengths of x (allowed multi-indices) and of the svec of y."""
    nx, ny = ctypes.c_int64(0), ctypes.c_int64(0)
    check(lib().psd_affine_dims(d, ctypes.byref(nx), ctypes.byref(ny)), "psd_affine_dims")
    return int(nx.value), int(ny.value)


def scs_workspace_size(settings: "ScsSettings", nbatch: int = 1) -> int:
    out = ctypes.c_size_t(0)
    check(lib().psd_scs_workspace_size_batched(ctypes.byref(settings), nbatch, ctypes.byref(out)),
          "psd_scs_workspace_size_batched")
    return int(out.value)


def affine_workspace_size(d: int) -> int:
    out = ctypes.c_size_t(0)
    check(lib().psd_affine_workspace_size(d, ctypes.byref(out)), "psd_affine_workspace_size")
    return int(out.value)
