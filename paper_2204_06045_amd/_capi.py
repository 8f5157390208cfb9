"""ctypes marshalling for ``libqtn.so`` (declarations in ``include/qtn.h``).

Only argument conversion lives here; every step of the contraction runs in
the library's HIP kernels.  torch is imported before the library is loaded so
that both share one HIP runtime; torch supplies device memory and streams.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libqtn.so")

QTN_OK = 0
QTN_EINVAL = -1
QTN_ERANGE = -2
QTN_ENOMEM = -3
QTN_EDEVICE = -4
QTN_ESTATE = -5

QTN_C128 = 0
QTN_C64 = 1
QTN_MIXED = 2

NKERNELS = 5
K_FILL, K_BLOCK, K_WIDE, K_REDUCE, K_PERSISTENT = range(5)
KERNEL_NAMES = ("fill", "block", "wide", "reduce", "persistent")

# every symbol include/qtn.h declares
EXPORTS = (
    "qtn_network_build", "qtn_network_info", "qtn_order_minfill", "qtn_plan",
    "qtn_set_angles", "qtn_contract", "qtn_contract_batch",
    "qtn_batch_workspace", "qtn_autotune_batch", "qtn_contract_timed", "qtn_get_plan_stats",
    "qtn_angles_workspace", "qtn_contract_angles", "qtn_gradient_workspace",
    "qtn_energy_gradient",
    "qtn_bucket_widths", "qtn_slice_vars", "qtn_network_free", "qtn_last_error", "qtn_launch_log",
    "qtn_plan_order", "qtn_autotune", "qtn_tune_angles_workspace", "qtn_autotune_angles",
    "qtn_tune_log", "qtn_tune_picks", "qtn_set_tune_picks",
    "qtn_costmodel_create", "qtn_costmodel_params", "qtn_costmodel_normalization",
    "qtn_costmodel_workspace", "qtn_costmodel_train", "qtn_costmodel_predict",
    "qtn_costmodel_grad", "qtn_costmodel_adam_step", "qtn_apply_costmodel",
    "qtn_costmodel_free", "qtn_bucket_plan", "qtn_bucket_get_info", "qtn_bucket_contract",
    "qtn_bucket_contract_noalloc", "qtn_bucket_contract_timed", "qtn_bucket_free",
)
MLP_PARAMS = 5508
MLP_OUT = 4  # predicted variants: workgroup, streaming, generic, matrix form


class qtn_config(ctypes.Structure):
    _fields_ = [("max_levels", ctypes.c_int32), ("small_width", ctypes.c_int32),
                ("max_width", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("eager", ctypes.c_int32), ("lane_sum_bits", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("order_trials", ctypes.c_int32),
                ("executor", ctypes.c_int32), ("spin_limit", ctypes.c_int32),
                ("mixed_width", ctypes.c_int32), ("slice_width", ctypes.c_int32),
                ("order_weight", ctypes.c_int32), ("hybrid_width", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class qtn_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NKERNELS),
                ("launches", ctypes.c_int64 * NKERNELS),
                ("bytes", ctypes.c_double * NKERNELS),
                ("flops", ctypes.c_double * NKERNELS)]


class qtn_launch_rec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("group", ctypes.c_int32),
                ("n_groups", ctypes.c_int32), ("w", ctypes.c_int32), ("L", ctypes.c_int32),
                ("n_ops", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("n_units", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("cvt", ctypes.c_int32), ("knob", ctypes.c_int32),
                ("serial", ctypes.c_int32), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class qtn_tune_report(ctypes.Structure):
    _fields_ = [("n_groups", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("cand_ms", ctypes.c_double * 8), ("tuned_ms", ctypes.c_double),
                ("picks", ctypes.c_int32 * 8)]


class qtn_batch_tune_report(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("pick", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32 * 8), ("item_order", ctypes.c_int32 * 8),
                ("ms", ctypes.c_double * 8)]


class qtn_tune_pick(ctypes.Structure):
    _fields_ = [("edge", ctypes.c_int32), ("group", ctypes.c_int32), ("place", ctypes.c_int8),
                ("variant", ctypes.c_int8), ("rls", ctypes.c_int8), ("pad", ctypes.c_int8),
                ("shape", ctypes.c_uint32)]


class qtn_tune_rec(ctypes.Structure):
    _fields_ = [("features", ctypes.c_float * 16), ("ms", ctypes.c_double * 4)]


class qtn_plan_stats(ctypes.Structure):
    _fields_ = [("n_buckets", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("n_wide", ctypes.c_int64), ("max_width", ctypes.c_int32),
                ("width_hist", ctypes.c_int32 * 40), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double), ("paper_flops", ctypes.c_double),
                ("workspace", ctypes.c_size_t), ("n_matrix", ctypes.c_int64),
                ("n_cell", ctypes.c_int64), ("n_stream", ctypes.c_int64),
                ("n_over4g", ctypes.c_int64), ("n_over4g_generic", ctypes.c_int64),
                ("n_sliced", ctypes.c_int64), ("n_slices", ctypes.c_int64)]


class qtn_bucket_info(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("L", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("knob", ctypes.c_int32),
                ("serial", ctypes.c_int32), ("n_units", ctypes.c_int64),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t), ("data_bytes", ctypes.c_int64)]


class QtnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"qtn error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            raise ImportError(
                f"{SO} is missing: build it with paper_2204_06045_amd/build.py "
                "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(SO)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        pi32 = ctypes.POINTER(ctypes.c_int32)
        pd = ctypes.POINTER(ctypes.c_double)
        L.qtn_last_error.restype = ctypes.c_char_p
        L.qtn_network_build.argtypes = [i32, i64, pi32, i32, pd, pd,
                                        ctypes.POINTER(qtn_config), ctypes.POINTER(P)]
        L.qtn_network_info.argtypes = [P, i64, pi32, pi32, pi32]
        L.qtn_order_minfill.argtypes = [P, i64, pi32]
        L.qtn_plan.argtypes = [P, ctypes.POINTER(pi32), i32,
                               ctypes.POINTER(ctypes.c_size_t)]
        L.qtn_set_angles.argtypes = [P, pd, pd]
        L.qtn_contract.argtypes = [P, P, ctypes.c_size_t, P, pd, pd, pd]
        L.qtn_contract_batch.argtypes = [ctypes.POINTER(P), i32, P, ctypes.c_size_t,
                                         P, pd, pd]
        L.qtn_batch_workspace.argtypes = [ctypes.POINTER(P), i32,
                                          ctypes.POINTER(ctypes.c_size_t)]
        L.qtn_autotune_batch.argtypes = [ctypes.POINTER(P), i32, P, ctypes.c_size_t, P,
                                         ctypes.POINTER(qtn_batch_tune_report)]
        L.qtn_contract_timed.argtypes = [P, P, ctypes.c_size_t, P, pd, pd,
                                         ctypes.POINTER(qtn_timing)]
        L.qtn_get_plan_stats.argtypes = [P, ctypes.POINTER(qtn_plan_stats)]
        L.qtn_bucket_widths.argtypes = [P, i64, pi32]
        L.qtn_slice_vars.argtypes = [P, i64, i32, pi32, pi32]
        L.qtn_plan_order.argtypes = [P, i64, pi32]
        L.qtn_autotune.argtypes = [P, P, ctypes.c_size_t, P, ctypes.POINTER(qtn_tune_report)]
        L.qtn_tune_angles_workspace.argtypes = [P, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.qtn_autotune_angles.argtypes = [P, P, ctypes.c_size_t, P, i32,
                                          ctypes.POINTER(qtn_tune_report)]
        L.qtn_tune_log.argtypes = [P, i64, ctypes.POINTER(qtn_tune_rec), ctypes.POINTER(i64)]
        L.qtn_angles_workspace.argtypes = [P, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.qtn_gradient_workspace.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.qtn_energy_gradient.argtypes = [P, P, ctypes.c_size_t, P, pd, pd, ctypes.c_double,
                                          pd, pd, pd]
        L.qtn_contract_angles.argtypes = [P, P, ctypes.c_size_t, P, i32, pd, pd, pd, pd,
                                          ctypes.POINTER(qtn_timing)]
        L.qtn_tune_picks.argtypes = [P, i64, ctypes.POINTER(qtn_tune_pick), ctypes.POINTER(i64)]
        L.qtn_set_tune_picks.argtypes = [P, ctypes.POINTER(qtn_tune_pick), i64]
        pf = ctypes.POINTER(ctypes.c_float)
        sz = ctypes.c_size_t
        L.qtn_costmodel_create.argtypes = [pf, ctypes.POINTER(P)]
        L.qtn_costmodel_params.argtypes = [P, pf]
        L.qtn_costmodel_normalization.argtypes = [P, pf, pf]
        L.qtn_costmodel_workspace.argtypes = [i64, ctypes.POINTER(sz)]
        L.qtn_costmodel_train.argtypes = [P, pf, pd, i64, i32, ctypes.c_float, P, sz, P, pf]
        L.qtn_costmodel_predict.argtypes = [P, pf, i64, P, sz, P, pf]
        L.qtn_costmodel_grad.argtypes = [P, pf, pf, pf, i64, P, sz, P, pf, pf]
        L.qtn_costmodel_adam_step.argtypes = [P, pf, ctypes.c_float, P, sz, P]
        L.qtn_apply_costmodel.argtypes = [P, P, P, sz, P, pi32]
        L.qtn_costmodel_free.argtypes = [P]
        L.qtn_costmodel_free.restype = None
        L.qtn_launch_log.argtypes = [P, i64, ctypes.POINTER(qtn_launch_rec),
                                     ctypes.POINTER(i64)]
        L.qtn_network_free.argtypes = [P]
        L.qtn_network_free.restype = None
        pi64 = ctypes.POINTER(ctypes.c_int64)
        L.qtn_bucket_plan.argtypes = [i32, pi32, pi32, pi64, i32, pi32, i64, i32, i32, i32,
                                      ctypes.POINTER(P)]
        L.qtn_bucket_get_info.argtypes = [P, ctypes.POINTER(qtn_bucket_info)]
        L.qtn_bucket_contract.argtypes = [P, P, sz, P, sz, P]
        L.qtn_bucket_contract_noalloc.argtypes = [P, P, sz, P]
        L.qtn_bucket_contract_timed.argtypes = [P, P, sz, P, sz, P, pd]
        L.qtn_bucket_free.argtypes = [P]
        L.qtn_bucket_free.restype = None
        for name in EXPORTS:
            if name not in ("qtn_network_free", "qtn_last_error", "qtn_costmodel_free",
                            "qtn_bucket_free"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc):
    if rc != QTN_OK:
        raise QtnError(rc, lib().qtn_last_error().decode())
    return rc
