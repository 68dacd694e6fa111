"""The paper's multithreaded scan on the host CPU (context beside the GPU path
and the sequential oracle; the GPU library never calls it).

cpu_two_pass_scan_u32 runs the Accumulate + Prefix Sum scheme with
cache-friendly partitions and one counting barrier per iteration (Sections
2.1-2.2 of the paper), built from two_pass_scan.c with gcc."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "two_pass_scan.c")
_LIB = os.path.join(_HERE, "libcpu_two_pass.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-pthread", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.cpu_two_pass_scan_u32.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int,
                                              ctypes.c_int64]
        lib.cpu_two_pass_scan_u32.restype = ctypes.c_int
        _lib = lib
    return _lib


def two_pass_scan_u32(a: np.ndarray, threads: int, partition: int, out: np.ndarray | None = None) -> np.ndarray:
    """Inclusive scan of 32-bit integers (wrapping), out may be a (in place)."""
    src = np.ascontiguousarray(a)
    if src.dtype not in (np.uint32, np.int32):
        raise TypeError("int32 / uint32 only")
    dst = np.empty_like(src) if out is None else out
    if _load().cpu_two_pass_scan_u32(src.ctypes.data, dst.ctypes.data, src.size, int(threads), int(partition)) != 0:
        raise RuntimeError("cpu_two_pass_scan_u32 failed")
    return dst
