"""ctypes binding of the C ABI in include/qtn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libqtn.so")

QTN_OK, QTN_EINVAL, QTN_ENOMEM, QTN_EDEVICE, QTN_EUNSUPPORTED, QTN_ESTATE = range(6)
QTN_C64, QTN_C128 = 0, 1
QTN_ORDER_MIN_DEGREE, QTN_ORDER_MIN_FILL = 0, 1
QTN_PLAIN, QTN_BATCHED = 0, 1
QTN_HOST_ONLY = -1
QTN_SCRATCH_BYTES = 64 << 20

STATUS_NAMES = {0: "QTN_OK", 1: "QTN_EINVAL", 2: "QTN_ENOMEM", 3: "QTN_EDEVICE", 4: "QTN_EUNSUPPORTED",
                5: "QTN_ESTATE"}

EXPORTS = [
    "qtn_create", "qtn_destroy", "qtn_last_error", "qtn_build", "qtn_order", "qtn_order_rgreedy",
    "qtn_workspace_size",
    "qtn_set_params", "qtn_contract", "qtn_energy_grad", "qtn_edge_results", "qtn_get_info",
    "qtn_cone_stats", "qtn_validate_plan", "qtn_get_tuning", "qtn_set_tuning", "qtn_autotune",
    "qtn_kernel_time", "qtn_set_sweep_timing", "qtn_gemm_census", "qtn_time_wide_ops", "qtn_set_memory_budget", "qtn_copy_bandwidth", "qtn_time_persistent",
    "qtn_build_amplitude", "qtn_amplitude", "qtn_cost_model", "qtn_cost_model_order", "qtn_energy_grad_noalloc",
    "qtn_time_wide_sweep", "qtn_get_band_tuning", "qtn_set_band_tuning", "qtn_autotune_bands",
    "qtn_net_free",
]


class QtnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("lane_cap", C.c_int32), ("seq_max_bits", C.c_int32),
                ("tile_blocks", C.c_int32), ("loop_cap", C.c_int32), ("grid", C.c_int32),
                ("lds_kb", C.c_int32), ("par_bits", C.c_int32), ("merge_bits", C.c_int32),
                ("merge_lam_bits", C.c_int32), ("lane_low", C.c_int32),
                ("fuse_adjoint", C.c_int32), ("lds_threads", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


QTN_BANDS = 3


class BandTuning(C.Structure):
    _fields_ = [("par_bits", C.c_int32), ("tile_blocks", C.c_int32), ("loop_cap", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Cost(C.Structure):
    _fields_ = [("n_indices", C.c_int32), ("n_tensors", C.c_int32), ("width", C.c_int32),
                ("log2_ops", C.c_double), ("order_seconds", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Info(C.Structure):
    _fields_ = [("n_cones", C.c_int32), ("p", C.c_int32), ("max_width", C.c_int32), ("dtype", C.c_int32),
                ("n_buckets", C.c_int64), ("n_ops_fwd", C.c_int64), ("n_ops_grad", C.c_int64),
                ("n_items_fwd", C.c_int64), ("n_items_grad", C.c_int64), ("fwd_bytes", C.c_double),
                ("bwd_bytes", C.c_double), ("fwd_flops", C.c_double), ("ws_fwd", C.c_size_t),
                ("ws_grad", C.c_size_t), ("n_lds_cones", C.c_int32), ("lds_window", C.c_int32),
                ("n_recomputed", C.c_int64), ("rec_bytes", C.c_double), ("arena_keep_all", C.c_size_t),
                ("n_steps", C.c_int64), ("fwd_bytes_bucket", C.c_double), ("bwd_bytes_bucket", C.c_double),
                ("pinned_bytes", C.c_size_t), ("max_cone_dynamic", C.c_size_t)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Loads the built library; raises if it has not been built (there is no
    fallback: every contraction runs in the HIP kernels of this library)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc for gfx950) first")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, SZ, D = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    sig = {
        "qtn_create": (I32, [C.c_int, C.POINTER(P)]),
        "qtn_destroy": (None, [P]),
        "qtn_last_error": (C.c_char_p, []),
        "qtn_build": (I32, [P, I32, I32, P, I32, I32, C.POINTER(P)]),
        "qtn_order": (I32, [P, I32, C.POINTER(I32)]),
        "qtn_order_rgreedy": (I32, [P, I32, I32, D, C.c_uint64, C.POINTER(I32)]),
        "qtn_workspace_size": (I32, [P, I32, C.POINTER(SZ)]),
        "qtn_set_params": (I32, [P, P, P]),
        "qtn_contract": (I32, [P, I32, P, SZ, P, P, P]),
        "qtn_energy_grad": (I32, [P, I32, P, SZ, P, P, P, P, P]),
        "qtn_edge_results": (I32, [P, P, P, P, P]),
        "qtn_get_info": (I32, [P, C.POINTER(Info)]),
        "qtn_cone_stats": (I32, [P, P, P, P, P, P, P, P]),
        "qtn_validate_plan": (I32, [P]),
        "qtn_get_tuning": (I32, [P, C.POINTER(Tuning)]),
        "qtn_set_tuning": (I32, [P, C.POINTER(Tuning)]),
        "qtn_autotune": (I32, [P, I32, P, SZ, P, I32, C.POINTER(Tuning)]),
        "qtn_kernel_time": (I32, [P, C.POINTER(D), C.POINTER(I64), I32]),
        "qtn_set_sweep_timing": (I32, [P, I32]),
        "qtn_gemm_census": (I32, [P, I32, C.POINTER(I64), C.POINTER(I64), C.POINTER(D), C.POINTER(D)]),
        "qtn_set_memory_budget": (I32, [P, SZ]),
        "qtn_time_wide_ops": (I32, [P, I32, I32, P, SZ, P, I32, C.POINTER(D), C.POINTER(D), C.POINTER(I64)]),
        "qtn_copy_bandwidth": (I32, [P, P, SZ, P, I32, C.POINTER(D)]),
        "qtn_time_persistent": (I32, [P, I32, P, SZ, P, I32, C.POINTER(D)]),
        "qtn_build_amplitude": (I32, [P, I32, I32, P, I32, I32, C.POINTER(P)]),
        "qtn_amplitude": (I32, [P, I32, P, SZ, P, P, P]),
        "qtn_cost_model": (I32, [I32, I32, P, I32, I32, I32, I32, D, C.c_uint64, C.POINTER(Cost)]),
        "qtn_cost_model_order": (I32, [I32, I32, P, I32, I32, I32, I32, D, C.c_uint64, C.POINTER(Cost), P, I32]),
        "qtn_energy_grad_noalloc": (I32, [P, I32, P, P, P, P, P]),
        "qtn_time_wide_sweep": (I32, [P, I32, I32, I32, I32, P, SZ, P, I32, C.POINTER(D), C.POINTER(D), C.POINTER(D),
                                      C.POINTER(I64), C.POINTER(I64)]),
        "qtn_get_band_tuning": (I32, [P, P]),
        "qtn_set_band_tuning": (I32, [P, P]),
        "qtn_autotune_bands": (I32, [P, I32, P, SZ, P, I32, P, C.POINTER(D)]),
        "qtn_net_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int) -> None:
    if status != QTN_OK:
        raise QtnError(status, lib().qtn_last_error().decode(errors="replace"))
