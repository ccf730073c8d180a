"""ctypes binding of libspiir.so (the C ABI declared in include/spiir.h).

Argument marshalling only: every step of the filtering runs in the library's
HIP kernels. Functions keep the C names; device buffers are passed as raw
pointers (``tensor.data_ptr()``) and streams as ``hipStream_t`` handles.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspiir.so")

SPIIR_OK, SPIIR_EINVAL, SPIIR_ENOMEM, SPIIR_EHIP, SPIIR_ESTATE, SPIIR_ENODEV = 0, -1, -2, -3, -4, -5
PREC_HYBRID, PREC_FP32, PREC_FP64_CARRY = 0, 1, 2

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = (
    "spiir_bank_opts_default", "spiir_bank_create", "spiir_bank_destroy", "spiir_bank_get_info",
    "spiir_bank_reset", "spiir_bank_set_coeffs", "spiir_bank_state_size", "spiir_bank_get_state",
    "spiir_bank_set_state", "spiir_filter_block", "spiir_trigger_max",
    "spiir_trigger_max_per_template", "spiir_forward_z", "spiir_backward", "spiir_tape_destroy",
    "spiir_batch_create", "spiir_batch_step", "spiir_batch_steps_total", "spiir_batch_reset",
    "spiir_batch_destroy", "spiir_batch_set_time_split", "spiir_autotune", "spiir_bank_time_kernels",
    "spiir_bank_kernel_time", "spiir_cluster_workspace_size", "spiir_cluster_triggers",
    "spiir_filter_block_z", "spiir_multirate_create", "spiir_multirate_destroy", "spiir_multirate_reset",
    "spiir_multirate_filter_block_z", "spiir_multirate_trigger_max", "spiir_multirate_level_bank",
    "spiir_multirate_set_graph",
    "spiir_whitener_create", "spiir_whitener_destroy", "spiir_whitener_estimate_psd", "spiir_whitener_set_psd",
    "spiir_whitener_get_psd", "spiir_whitener_process", "spiir_whitener_reset",
    "spiir_trigger_stream_create", "spiir_trigger_stream_push", "spiir_trigger_stream_flush",
    "spiir_trigger_stream_reset", "spiir_trigger_stream_destroy",
    "spiir_trigger_max_noalloc", "spiir_bank_set_coeffs_dev",
    "spiir_last_error", "spiir_version",
)


class SpiirError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__("%s failed (%d): %s" % (func, code, msg))
        self.code = code


class BankOpts(ctypes.Structure):
    _fields_ = [("chunk_len", ctypes.c_int32), ("filters_per_lane", ctypes.c_int32),
                ("max_delay", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("max_block", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("time_split", ctypes.c_int32), ("delay_band", ctypes.c_int32)]


class BankInfo(ctypes.Structure):
    _fields_ = [("n_templates", ctypes.c_int32), ("n_filters", ctypes.c_int64),
                ("max_delay", ctypes.c_int32), ("chunk_len", ctypes.c_int32),
                ("filters_per_lane", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("n_groups", ctypes.c_int32), ("n_slots", ctypes.c_int64),
                ("lds_bytes", ctypes.c_int32), ("x_in_lds", ctypes.c_int32),
                ("sub_block", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("n_cu", ctypes.c_int32), ("time_split", ctypes.c_int32),
                ("n_parts", ctypes.c_int32), ("delay_band", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load():
    """Loads libspiir.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libspiir.so is not built; run __graft_entry__.build() "
                           "or python paper_1602_05573_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "spiir_bank_opts_default": (None, [ctypes.POINTER(BankOpts)]),
        "spiir_bank_create": (ctypes.c_int, [PP, I32, P, P, P, P, ctypes.POINTER(BankOpts)]),
        "spiir_bank_destroy": (ctypes.c_int, [P]),
        "spiir_bank_get_info": (ctypes.c_int, [P, ctypes.POINTER(BankInfo)]),
        "spiir_bank_reset": (ctypes.c_int, [P, P]),
        "spiir_bank_set_coeffs": (ctypes.c_int, [P, P, P]),
        "spiir_bank_set_coeffs_dev": (ctypes.c_int, [P, P, P, P]),
        "spiir_bank_state_size": (ctypes.c_int, [P, ctypes.POINTER(SZ)]),
        "spiir_bank_get_state": (ctypes.c_int, [P, P, SZ]),
        "spiir_bank_set_state": (ctypes.c_int, [P, P, SZ]),
        "spiir_filter_block": (ctypes.c_int, [P, P, I64, P, I64, P]),
        "spiir_trigger_max": (ctypes.c_int, [P, P, I64, P, P, P]),
        "spiir_trigger_max_noalloc": (ctypes.c_int, [P, P, I64, P, P, P]),
        "spiir_trigger_max_per_template": (ctypes.c_int, [P, P, I64, P, P, P, P]),
        "spiir_forward_z": (ctypes.c_int, [P, P, I64, P, PP, P]),
        "spiir_backward": (ctypes.c_int, [P, P, P, P, P, P]),
        "spiir_tape_destroy": (ctypes.c_int, [P]),
        "spiir_batch_create": (ctypes.c_int, [PP, I32, P, P, P, P, P, I32, P]),
        "spiir_batch_step": (ctypes.c_int, [P, P]),
        "spiir_batch_steps_total": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
        "spiir_batch_reset": (ctypes.c_int, [P, P]),
        "spiir_batch_destroy": (ctypes.c_int, [P]),
        "spiir_batch_set_time_split": (ctypes.c_int, [P, I32]),
        "spiir_autotune": (ctypes.c_int, [I32, P, P, P, P, P, I32, I32, I32,
                                          ctypes.POINTER(I32), ctypes.POINTER(I32), P]),
        "spiir_bank_time_kernels": (ctypes.c_int, [P, I32]),
        "spiir_bank_kernel_time": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]),
        "spiir_cluster_workspace_size": (ctypes.c_int, [I64, ctypes.POINTER(SZ)]),
        "spiir_cluster_triggers": (ctypes.c_int, [P, P, I64, ctypes.c_float, I32, P, SZ, P, P, P, I64,
                                                  P, I32, P]),
        "spiir_filter_block_z": (ctypes.c_int, [P, P, I64, P, I64, P]),
        "spiir_multirate_create": (ctypes.c_int, [PP, I32, I32, P, P, P, P, P, I32, P, I32,
                                                  ctypes.POINTER(BankOpts)]),
        "spiir_multirate_destroy": (ctypes.c_int, [P]),
        "spiir_multirate_reset": (ctypes.c_int, [P, P]),
        "spiir_multirate_filter_block_z": (ctypes.c_int, [P, P, I64, P, I64, P]),
        "spiir_multirate_trigger_max": (ctypes.c_int, [P, P, I64, P, P, P]),
        "spiir_multirate_level_bank": (ctypes.c_int, [P, I32, PP]),
        "spiir_multirate_set_graph": (ctypes.c_int, [P, I32]),
        "spiir_whitener_create": (ctypes.c_int, [PP, I32, I32, I32]),
        "spiir_whitener_destroy": (ctypes.c_int, [P]),
        "spiir_whitener_estimate_psd": (ctypes.c_int, [P, P, I64, P]),
        "spiir_whitener_set_psd": (ctypes.c_int, [P, P]),
        "spiir_whitener_get_psd": (ctypes.c_int, [P, P]),
        "spiir_whitener_process": (ctypes.c_int, [P, P, I64, P, P]),
        "spiir_whitener_reset": (ctypes.c_int, [P, P]),
        "spiir_trigger_stream_create": (ctypes.c_int, [PP, ctypes.c_float, I32, I64, I32]),
        "spiir_trigger_stream_push": (ctypes.c_int, [P, P, P, I64, P, P, P, I64, P, P]),
        "spiir_trigger_stream_flush": (ctypes.c_int, [P, P, P, P, I64, P, P]),
        "spiir_trigger_stream_reset": (ctypes.c_int, [P, P]),
        "spiir_trigger_stream_destroy": (ctypes.c_int, [P]),
        "spiir_last_error": (ctypes.c_char_p, []),
        "spiir_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, func: str):
    if rc != SPIIR_OK:
        msg = load().spiir_last_error().decode(errors="replace")
        raise SpiirError(rc, func, msg)


def call(name: str, *args):
    """Calls a status-returning function by its C name and raises on failure."""
    rc = getattr(load(), name)(*args)
    check(rc, name)
    return rc


def default_opts() -> BankOpts:
    o = BankOpts()
    load().spiir_bank_opts_default(ctypes.byref(o))
    return o
