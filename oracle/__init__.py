"""Sequential CPU oracle for the prefix-sum hot path (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this package, and this package imports nothing from the product.

Every routine follows the scan definition of the paper's Introduction
(inclusive: out[i] = a[0] + ... + a[i]; exclusive: identity first, last total
dropped) computed by the basic algorithm described there -- one sequential pass
of additions.  The arithmetic lives in ``scan_oracle.c`` (plain C99, built with
gcc -O2, no fast-math); this module only marshals numpy arrays.

Readings of points the paper leaves open (wrap-around for 32-bit integers,
float32 accumulated in float64, reverse and segmented forms) are documented in
``scan_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "scan_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_scan.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile scan_oracle.c into liboracle_scan.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
             "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        lib.oracle_scan_u32.argtypes = [P, P, I64, I, I]
        lib.oracle_scan_f32_f64.argtypes = [P, P, P, I64, I, I]
        lib.oracle_segmented_u32.argtypes = [P, P, P, I64, I, I]
        lib.oracle_segmented_f32_f64.argtypes = [P, P, P, P, I64, I, I]
        lib.oracle_scan_op_u32.argtypes = [P, P, I64, I, I, I, I]
        lib.oracle_segmented_op_u32.argtypes = [P, P, P, I64, I, I, I, I]
        lib.oracle_compact_u32.argtypes = [P, P, I64, I, I, ctypes.c_uint32]
        lib.oracle_compact_u32.restype = I64
        lib.oracle_scan_u64.argtypes = [P, P, I64, I, I]
        lib.oracle_scan_u64.restype = None
        lib.oracle_partition_u32.argtypes = [P, P, I64, I, I, ctypes.c_uint32]
        lib.oracle_partition_u32.restype = I64
        lib.oracle_scan_f64.argtypes = [P, P, P, I64, I, I]
        lib.oracle_scan_f64.restype = None
        for f in (lib.oracle_scan_u32, lib.oracle_scan_f32_f64,
                  lib.oracle_segmented_u32, lib.oracle_segmented_f32_f64,
                  lib.oracle_scan_op_u32, lib.oracle_segmented_op_u32):
            f.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _as_u32(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype not in (np.uint32, np.int32):
        raise TypeError("integer oracle takes int32/uint32, got %s" % a.dtype)
    return a.view(np.uint32)


def scan_int(a: np.ndarray, exclusive: bool = False, reverse: bool = False,
             out: np.ndarray | None = None) -> np.ndarray:
    """Scan of 32-bit integers, wrapping modulo 2^32.

    Returns an array of a's dtype (int32 stays int32: two's complement bits).
    ``out`` may be ``a`` itself (in place).
    """
    src = _as_u32(a)
    dst = np.empty_like(src) if out is None else _as_u32(out)
    _load().oracle_scan_u32(_ptr(src), _ptr(dst), src.size, int(exclusive), int(reverse))
    return dst.view(np.asarray(a).dtype)


def scan_int64(a: np.ndarray, exclusive: bool = False, out: np.ndarray | None = None,
               reverse: bool = False) -> np.ndarray:
    """Scan of 64-bit integers, wrapping modulo 2^64 (reverse: suffix scan).

    Returns an array of a's dtype (int64 or uint64); ``out`` may be ``a``.
    """
    a = np.ascontiguousarray(a)
    if a.dtype not in (np.uint64, np.int64):
        raise TypeError("64-bit oracle takes int64/uint64, got %s" % a.dtype)
    src = a.view(np.uint64)
    dst = np.empty_like(src) if out is None else out.view(np.uint64)
    _load().oracle_scan_u64(_ptr(src), _ptr(dst), src.size, int(exclusive), int(reverse))
    return dst.view(a.dtype)


def scan_f64(a: np.ndarray, exclusive: bool = False, with_abs: bool = True, reverse: bool = False):
    """Prefix sums (reverse: suffix sums) of float64 input, accumulated in
    double-double and rounded once to float64.

    Returns (sums, abs_sums): float64 arrays; abs_sums[i] is the running sum
    of |a| (the scale of the error tolerance), or None if ``with_abs`` is False.
    """
    src = np.ascontiguousarray(a, dtype=np.float64)
    s = np.empty(src.size, dtype=np.float64)
    ab = np.empty(src.size, dtype=np.float64) if with_abs else None
    _load().oracle_scan_f64(_ptr(src), _ptr(s), _ptr(ab), src.size, int(exclusive), int(reverse))
    return s, ab


def f64_tolerance(abs_sums: np.ndarray, depth: int) -> np.ndarray:
    """Per-element float64 acceptance bound for a sum evaluated by a tree of
    additions at most `depth` deep: depth * 2^-53 * (running sum of |a|), plus
    one rounding of the result (the standard bound for recursive summation)."""
    return np.ldexp(abs_sums, -53) * (depth + 1) * (1 + 1e-6)


def scan_f32(a: np.ndarray, exclusive: bool = False, reverse: bool = False,
             with_abs: bool = True):
    """Sequential float64 scan of float32 input.

    Returns (sums, abs_sums): float64 arrays; abs_sums[i] is the same scan over
    |a| (the scale of the error tolerance), or None if ``with_abs`` is False.
    """
    src = np.ascontiguousarray(a, dtype=np.float32)
    s = np.empty(src.size, dtype=np.float64)
    ab = np.empty(src.size, dtype=np.float64) if with_abs else None
    _load().oracle_scan_f32_f64(_ptr(src), _ptr(s), _ptr(ab), src.size,
                                int(exclusive), int(reverse))
    return s, ab


def _check_offsets(offsets: np.ndarray, n: int) -> np.ndarray:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if off.ndim != 1 or off.size < 1:
        raise ValueError("offsets must be a 1-D array of S+1 entries")
    if off[0] != 0 or off[-1] != n or np.any(np.diff(off) < 0):
        raise ValueError("offsets must start at 0, end at n and not decrease")
    return off


def segmented_int(a: np.ndarray, offsets: np.ndarray, exclusive: bool = False,
                  reverse: bool = False) -> np.ndarray:
    """Per-segment scan of 32-bit integers (restart at every segment start)."""
    src = _as_u32(a)
    off = _check_offsets(offsets, src.size)
    dst = np.empty_like(src)
    _load().oracle_segmented_u32(_ptr(src), _ptr(dst), _ptr(off), off.size - 1,
                                 int(exclusive), int(reverse))
    return dst.view(np.asarray(a).dtype)


def segmented_f32(a: np.ndarray, offsets: np.ndarray, exclusive: bool = False,
                  reverse: bool = False, with_abs: bool = True):
    """Per-segment sequential float64 scan of float32 input."""
    src = np.ascontiguousarray(a, dtype=np.float32)
    off = _check_offsets(offsets, src.size)
    s = np.empty(src.size, dtype=np.float64)
    ab = np.empty(src.size, dtype=np.float64) if with_abs else None
    _load().oracle_segmented_f32_f64(_ptr(src), _ptr(s), _ptr(ab), _ptr(off),
                                     off.size - 1, int(exclusive), int(reverse))
    return s, ab


OPERATORS = {"max": 1, "min": 2, "xor": 3}


def scan_op(a: np.ndarray, op: str, exclusive: bool = False, reverse: bool = False) -> np.ndarray:
    """Scan of 32-bit integers with another associative operator of the
    Introduction's definition: "max", "min" (signed for int32, unsigned for
    uint32) or "xor"; the exclusive form starts from the operator's identity."""
    src = _as_u32(a)
    dst = np.empty_like(src)
    _load().oracle_scan_op_u32(_ptr(src), _ptr(dst), src.size, OPERATORS[op],
                               int(np.asarray(a).dtype == np.int32), int(exclusive), int(reverse))
    return dst.view(np.asarray(a).dtype)


def segmented_op(a: np.ndarray, offsets: np.ndarray, op: str, exclusive: bool = False,
                 reverse: bool = False) -> np.ndarray:
    """Per-segment scan_op (restart from the identity at every segment start)."""
    src = _as_u32(a)
    off = _check_offsets(offsets, src.size)
    dst = np.empty_like(src)
    _load().oracle_segmented_op_u32(_ptr(src), _ptr(dst), _ptr(off), off.size - 1, OPERATORS[op],
                                    int(np.asarray(a).dtype == np.int32), int(exclusive), int(reverse))
    return dst.view(np.asarray(a).dtype)


PREDICATES = {"nonzero": 0, "greater": 1}


def compact(a: np.ndarray, predicate: str = "nonzero", threshold=0) -> np.ndarray:
    """The elements of a (int32 / uint32 / float32) that the predicate keeps,
    in order: "nonzero" (32 bits not all zero) or "greater" (x > threshold in
    a's type; NaN never kept)."""
    a = np.ascontiguousarray(a)
    dt = {np.dtype(np.int32): 0, np.dtype(np.uint32): 1, np.dtype(np.float32): 2}[a.dtype]
    thr = np.array([threshold], dtype=a.dtype).view(np.uint32)[0]
    src = a.view(np.uint32)
    dst = np.empty_like(src)
    k = _load().oracle_compact_u32(_ptr(src), _ptr(dst), src.size, PREDICATES[predicate], dt, int(thr))
    return dst[:k].view(a.dtype).copy()


def partition(a: np.ndarray, predicate: str = "nonzero", threshold=0):
    """Two-way partition of a (int32 / uint32 / float32) by the predicate of
    compact: returns (out, k) with the kept elements in out[:k] in input order
    and the others in out[k:] in reverse input order."""
    a = np.ascontiguousarray(a)
    dt = {np.dtype(np.int32): 0, np.dtype(np.uint32): 1, np.dtype(np.float32): 2}[a.dtype]
    thr = np.array([threshold], dtype=a.dtype).view(np.uint32)[0]
    src = a.view(np.uint32)
    dst = np.empty_like(src)
    k = _load().oracle_partition_u32(_ptr(src), _ptr(dst), src.size, PREDICATES[predicate], dt, int(thr))
    return dst.view(a.dtype), int(k)


def f32_tolerance(abs_sums: np.ndarray) -> np.ndarray:
    """Per-element float32 acceptance bound: 2^-20 times the running sum of |a|."""
    return np.ldexp(abs_sums, -20)
