"""ctypes binding of libmi355scan.so (argument marshalling only).

The library is required: importing this module without the built library
raises ImportError -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

# torch ships its own HIP runtime with the same soname as /opt/rocm's.  Import
# it first so the library below binds to the runtime torch already uses: two
# HIP runtimes in one process would not share devices, streams or memory.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmi355scan.so")

SCAN_I32, SCAN_U32, SCAN_F32, SCAN_I64, SCAN_U64, SCAN_F64 = 0, 1, 2, 3, 4, 5
SCAN_EXCLUSIVE, SCAN_REVERSE = 0x1, 0x2
SCAN_TWO_PASS_PREFIX_INCREMENT, SCAN_TWO_PASS_ACCUMULATE_PREFIX = 0, 1
SCAN_PRED_NONZERO, SCAN_PRED_GREATER = 0, 1

STATUS_NAMES = {
    0: "SCAN_SUCCESS", 1: "SCAN_ERROR_INVALID_VALUE", 2: "SCAN_ERROR_OVERLAP",
    3: "SCAN_ERROR_OUT_OF_MEMORY", 4: "SCAN_ERROR_LAUNCH", 5: "SCAN_ERROR_NOT_SUPPORTED",
    6: "SCAN_ERROR_CAPTURE", 7: "SCAN_ERROR_TIMEOUT",
}

P = ctypes.c_void_p
I32 = ctypes.c_int32
U32 = ctypes.c_uint32
I64 = ctypes.c_int64
ST = ctypes.c_int

# name -> (restype, argtypes); mirrors include/mi355scan.h
SIGNATURES = {
    "scan_inclusive_i32": (ST, [P, P, I64, P]),
    "scan_inclusive_u32": (ST, [P, P, I64, P]),
    "scan_inclusive_f32": (ST, [P, P, I64, P]),
    "scan_exclusive_i32": (ST, [P, P, I64, P]),
    "scan_exclusive_u32": (ST, [P, P, I64, P]),
    "scan_exclusive_f32": (ST, [P, P, I64, P]),
    "scan_flat": (ST, [P, P, I64, ST, U32, P]),
    "scan_flat_noalloc": (ST, [P, P, I64, ST, U32, P]),
    "scan_stream_ceiling": (ST, [P, P, I64, I32, P]),
    "scan_segmented_batch": (ST, [P, P, P, I32, I64, ST, U32, P]),
    "scan_two_pass": (ST, [P, P, I64, ST, U32, I32, I64, P]),
    "scan_compact": (ST, [P, P, I64, ST, I32, U32, P, P]),
    "scan_partition": (ST, [P, P, I64, ST, I32, U32, P, P]),
    "scan_f32_backward": (ST, [P, P, I64, P, I32, P]),
    "scan_reserve": (ST, [I64, P]),
    "scan_release": (ST, [P]),
    "scan_segmented_graph_create": (ST, [P, P, P, I32, I64, ST, U32, P, ctypes.POINTER(P)]),
    "scan_looped_graph_create": (ST, [P, P, P, I32, ST, U32, P, ctypes.POINTER(P)]),
    "scan_graph_launch": (ST, [P, P]),
    "scan_graph_check_device_error": (ST, [P]),
    "scan_graph_destroy": (ST, [P]),
    "scan_segmented_looped": (ST, [P, P, P, I32, ST, U32, P]),
    "scan_num_configs": (I32, []),
    "scan_config_info": (ST, [I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                              ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "scan_force_config": (ST, [I32]),
    "scan_selected_config": (I32, [ST, U32, I32, I64]),
    "scan_autotune": (ST, [P, P, I64, P, I32, ST, U32, I32, P, ctypes.POINTER(I32)]),
    "scan_tune_save": (ST, [ctypes.c_char_p]),
    "scan_tune_load": (ST, [ctypes.c_char_p]),
    "scan_status_string": (ctypes.c_char_p, [ST]),
    "scan_last_hip_error": (I32, []),
    "scan_set_spin_limit": (ST, [U32]),
    "scan_check_device_error": (ST, [P]),
}


class ScanError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        self.name = STATUS_NAMES.get(status, "unknown")
        msg = "%s failed: %s (%d)" % (what or "scan call", self.name, status)
        if status == 4:
            msg += ", hipError_t %d" % _lib.scan_last_hip_error()
        if status == 7:
            msg += (": a device-side wait of an earlier call on this stream (or graph) gave up, so that"
                    " call's results are invalid; this call enqueued nothing")
        super().__init__(msg)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("%s is not built (run `python -m paper_2312_14874_amd.build`)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
lib = _lib


def check(status: int, what: str = "") -> None:
    if status != 0:
        raise ScanError(status, what)
