"""ctypes binding to libpm.so (argument marshalling only).

Every function here forwards to the C ABI declared in include/pm.h; device
memory comes from torch tensors and streams from torch's current HIP stream.
The library must be built (``python -m paper_0802_2488_amd.build``); there is
no fallback of any kind when it is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("PM_LIB_PATH") or os.path.join(HERE, "libpm.so")

PM_OK, PM_EINVAL, PM_EDEVICE, PM_ENOCONV, PM_ENAN, PM_EBUSY = 0, -1, -3, -4, -5, -6
PM_FP32, PM_FP64 = 0, 1
PM_MAX_L = 8192


class PmParams(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("mu", ctypes.c_double), ("lam", ctypes.c_double), ("Y", ctypes.c_double),
        ("mu0", ctypes.c_double), ("lam0", ctypes.c_double),
        ("eta_eq", ctypes.c_double), ("eta_mac", ctypes.c_double), ("eta_cmp", ctypes.c_double),
        ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("green_variant", ctypes.c_int32),
    ]


class PmStepOut(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("plastic", ctypes.c_void_p),
        ("sigma_mean", ctypes.c_double * 4), ("eps_mean", ctypes.c_double * 4),
        ("res_eq", ctypes.c_double), ("res_mac", ctypes.c_double), ("res_cmp", ctypes.c_double),
        ("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
    ]


class PmKernelTiming(ctypes.Structure):
    _fields_ = [
        ("col_ms", ctypes.c_double), ("col_launches", ctypes.c_int64),
        ("row_ms", ctypes.c_double), ("row_launches", ctypes.c_int64),
        ("other_ms", ctypes.c_double), ("iterations", ctypes.c_int64),
    ]


class PmStepRecord(ctypes.Structure):
    _fields_ = [
        ("sigma_mean", ctypes.c_double * 4), ("eps_mean", ctypes.c_double * 4),
        ("res_eq", ctypes.c_double), ("res_mac", ctypes.c_double), ("res_cmp", ctypes.c_double),
        ("plastic_fraction", ctypes.c_double),
        ("iters", ctypes.c_int32), ("status", ctypes.c_int32),
    ]


class PmSlotInfo(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("precision", ctypes.c_int32), ("nsteps", ctypes.c_int32),
        ("steps_done", ctypes.c_int32), ("finished", ctypes.c_int32), ("last_status", ctypes.c_int32),
        ("held", ctypes.c_int32),
    ]


PM_STEP_CONVERGED, PM_STEP_NOCONV, PM_STEP_NAN = 1, 2, 3
PM_ADMIT_HOLD = 1


class PmTuneResult(ctypes.Structure):
    _fields_ = [("row_variant", ctypes.c_int32), ("col_variant", ctypes.c_int32),
                ("ms_per_iteration", (ctypes.c_double * 2) * 2)]


class PmClusterStats(ctypes.Structure):
    _fields_ = [
        ("n_void", ctypes.c_int64), ("n_plastic", ctypes.c_int64), ("n_void_clusters", ctypes.c_int64),
        ("n_clusters_raw", ctypes.c_int64), ("n_isolated_void_clusters", ctypes.c_int64),
        ("n_plastic_only_clusters", ctypes.c_int64), ("n_clusters", ctypes.c_int64), ("largest", ctypes.c_int64),
        ("largest_label", ctypes.c_int32), ("spans_x1", ctypes.c_int32), ("spans_x2", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class PmClusterIndicators(ctypes.Structure):
    _fields_ = [("v_p", ctypes.c_double), ("f_p", ctypes.c_double), ("v_max", ctypes.c_double),
                ("i", ctypes.c_double), ("n", ctypes.c_double)]


class PmStrainMapOut(ctypes.Structure):
    _fields_ = [("mean_eq", ctypes.c_double), ("max_eq", ctypes.c_double), ("checkerboard", ctypes.c_double),
                ("sharpness", ctypes.c_double), ("matrix_pixels", ctypes.c_int64)]


class PmDg2Out(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_void_p), ("sigma_of_avg", ctypes.c_void_p), ("sigma_avg", ctypes.c_void_p),
        ("plastic", ctypes.c_void_p),
        ("eps_mean", ctypes.c_double * 4), ("sigma_of_avg_mean", ctypes.c_double * 4),
        ("sigma_avg_mean", ctypes.c_double * 4), ("plastic_fraction", ctypes.c_double),
    ]

# (name, restype, argtypes) of every entry point in include/pm.h
SIGNATURES = [
    ("pm_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("pm_last_error", ctypes.c_char_p, []),
    ("pm_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(PmParams)]),
    ("pm_solver_create", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(PmParams), ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_size_t, ctypes.c_void_p]),
    ("pm_solver_step", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(PmStepOut)]),
    ("pm_solver_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("pm_solver_set_max_iter", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("pm_bernoulli_mask", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p]),
    ("pm_spectrum_tile", ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32]),
    ("pm_solver_buffers", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    ("pm_solver_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(PmKernelTiming)]),
    ("pm_debug_forward", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("pm_debug_inverse", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("pm_debug_green", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    ("pm_batch_overhead_bytes", ctypes.c_size_t, [ctypes.c_int32]),
    ("pm_batch_slot_bytes", ctypes.c_size_t, [ctypes.POINTER(PmParams), ctypes.c_int32]),
    ("pm_batch_create", ctypes.c_int,
     [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p]),
    ("pm_batch_admit", ctypes.c_int,
     [ctypes.c_void_p, ctypes.POINTER(PmParams), ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("pm_batch_resume", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("pm_batch_tick", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    ("pm_batch_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(PmSlotInfo)]),
    ("pm_batch_records", ctypes.c_int,
     [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(PmStepRecord)]),
    ("pm_batch_fetch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(PmStepOut)]),
    ("pm_batch_release", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("pm_batch_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("pm_batch_set_graphs", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("pm_cluster_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32]),
    ("pm_clusters", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
      ctypes.POINTER(PmClusterStats), ctypes.c_void_p]),
    ("pm_cluster_indicators", ctypes.c_int,
     [ctypes.POINTER(PmClusterStats), ctypes.c_int32, ctypes.c_double, ctypes.POINTER(PmClusterIndicators)]),
    ("pm_path_derivatives", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("pm_strain_map_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32]),
    ("pm_strain_map_metrics", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
      ctypes.POINTER(PmStrainMapOut), ctypes.c_void_p]),
    ("pm_five_point_average", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("pm_autotune_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    ("pm_autotune", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
      ctypes.POINTER(PmTuneResult)]),
    ("pm_set_tuning", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    ("pm_get_tuning", ctypes.c_int,
     [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("pm_dg2_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(PmParams)]),
    ("pm_dg2_combine", ctypes.c_int,
     [ctypes.POINTER(PmParams), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
      ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(PmDg2Out), ctypes.c_void_p]),
    ("pm_dg2_combine_static_max_bytes", ctypes.c_size_t, []),
    ("pm_dg2_combine_static", ctypes.c_int,
     [ctypes.POINTER(PmParams), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
      ctypes.POINTER(PmDg2Out), ctypes.c_void_p]),
]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libpm.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_0802_2488_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PmError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().pm_last_error().decode()
        super().__init__(f"{where}: {lib().pm_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def check(code: int, where: str) -> int:
    if code != PM_OK:
        raise PmError(code, where)
    return code
