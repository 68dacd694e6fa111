"""Seeded synthetic inputs for the scan workloads.

This module only draws random inputs; it holds none of the scan arithmetic.
Both sides of every parity check (the HIP library and the CPU oracle) receive
the same arrays from here.  Generators are numpy PCG64 streams seeded per
workload, so a given (workload, seed) always produces the same bytes.

Workloads (the paper's own experiments use random float32 data, 128 MB per
thread, in place -- Section 4.1; the shapes below are this library's test and
benchmark cases):

  small_i32      n = 2^20 int32, uniform in [0, 100)           (seed 1001)
  full_u32       n = 2^28 uint32, uniform over all 2^32 values  (seed 1002)
  normal_f32     n = 2^28 float32, i.i.d. normal(0, 1)          (seed 1003)
  segments       S = 4096 segments, lengths log-uniform in [1, 2^20],
                 int32 values Poisson(8)                        (seed 1004)
  rows           64 rows, lengths log-uniform in [2^10, 2^22],
                 x and upstream gradient normal(0, 1) float32   (seed 1005)
  fd_rows        16 rows of length 256, normal(0, 1) float32    (seed 1006)
"""
from __future__ import annotations

import numpy as np

SEEDS = {
    "small_i32": 1001,
    "full_u32": 1002,
    "normal_f32": 1003,
    "segments": 1004,
    "rows": 1005,
    "fd_rows": 1006,
}


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_i32(n: int, seed: int = SEEDS["small_i32"], lo: int = 0, hi: int = 100) -> np.ndarray:
    """int32 values uniform in [lo, hi)."""
    return rng(seed).integers(lo, hi, size=n, dtype=np.int32)


def full_u32(n: int, seed: int = SEEDS["full_u32"]) -> np.ndarray:
    """uint32 values uniform over the full 32-bit range (sums wrap constantly)."""
    return rng(seed).integers(0, 2**32, size=n, dtype=np.uint32)


def normal_f32(n: int, seed: int = SEEDS["normal_f32"]) -> np.ndarray:
    """float32 values i.i.d. normal(0, 1)."""
    return rng(seed).standard_normal(n, dtype=np.float32)


def small_int_f32(n: int, seed: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """float32 holding integers in [lo, hi]: every partial sum of n <= 2^22 of
    them is exactly representable, so every summation order gives the same
    bits."""
    return rng(seed).integers(lo, hi + 1, size=n).astype(np.float32)


def loguniform_lengths(g: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    """Integer lengths L = floor(exp(U(ln lo, ln(hi + 1)))), clamped to [lo, hi]."""
    u = g.uniform(np.log(lo), np.log(hi + 1), size=count)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def offsets_from_lengths(lengths: np.ndarray) -> np.ndarray:
    """CSR offsets (S + 1 int64 entries) of consecutive segments."""
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def segments(seed: int = SEEDS["segments"], num_segments: int = 4096,
             lo: int = 1, hi: int = 2**20, mean: float = 8.0):
    """Radix-histogram-like batch: (values int32 Poisson(mean), offsets int64)."""
    g = rng(seed)
    lengths = loguniform_lengths(g, num_segments, lo, hi)
    off = offsets_from_lengths(lengths)
    vals = g.poisson(mean, size=int(off[-1])).astype(np.int32)
    return vals, off


def rows(seed: int = SEEDS["rows"], num_rows: int = 64, lo: int = 2**10, hi: int = 2**22):
    """Ragged float32 rows: (x, upstream grad, offsets)."""
    g = rng(seed)
    lengths = loguniform_lengths(g, num_rows, lo, hi)
    off = offsets_from_lengths(lengths)
    n = int(off[-1])
    x = g.standard_normal(n, dtype=np.float32)
    gy = g.standard_normal(n, dtype=np.float32)
    return x, gy, off


def fd_rows(seed: int = SEEDS["fd_rows"], num_rows: int = 16, length: int = 256):
    """Fixed-length rows for the finite-difference gradient check: (x, g), shape (rows, length)."""
    g = rng(seed)
    x = g.standard_normal((num_rows, length), dtype=np.float32)
    gy = g.standard_normal((num_rows, length), dtype=np.float32)
    return x, gy


def random_offsets(g: np.random.Generator, n: int, num_segments: int, p_empty: float = 0.2) -> np.ndarray:
    """Random CSR offsets over n elements with some empty segments (for edge tests)."""
    if num_segments <= 0:
        raise ValueError("num_segments must be positive")
    cuts = np.sort(g.integers(0, n + 1, size=num_segments - 1))
    off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    # force some repeated cut points (empty segments)
    k = int(p_empty * (num_segments - 1))
    if k > 0 and num_segments > 2:
        idx = g.choice(np.arange(1, num_segments), size=k, replace=False)
        off[idx] = off[idx - 1]
        off = np.maximum.accumulate(off)
    return off
