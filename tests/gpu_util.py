"""Helpers shared by the GPU tests: move seeded numpy inputs to the device,
call the C ABI, bring results back.  No scan arithmetic here."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

DT = {np.dtype(np.int32): 0, np.dtype(np.uint32): 1, np.dtype(np.float32): 2}


def lib():
    import paper_2312_14874_amd as m
    return m.lib


def stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_dev(a: np.ndarray, pad: int = 0) -> torch.Tensor:
    """Device copy of a (uint32 stored as int32 bits), with `pad` spare
    elements in front so sub-pointers can be misaligned."""
    bits = a.view(np.int32) if a.dtype == np.uint32 else a
    t = torch.empty(a.size + pad, dtype=torch.float32 if a.dtype == np.float32 else torch.int32,
                    device="cuda")
    t[pad:].copy_(torch.from_numpy(np.ascontiguousarray(bits)))
    return t


def from_dev(t: torch.Tensor, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype)


def check_status(s, what="call"):
    assert s == 0, "%s returned %d (%s)" % (what, s, lib().scan_status_string(s))


def flat(a: np.ndarray, exclusive=False, reverse=False, inplace=False, misalign=0, cfg=None):
    """Run scan_flat on a copy of a; returns the numpy result."""
    L = lib()
    x = to_dev(a, pad=misalign + 4)
    xin = x[misalign + 4:]
    out = xin if inplace else torch.empty(a.size + misalign + 4, dtype=x.dtype, device="cuda")[misalign + 4:]
    if cfg is not None:
        check_status(L.scan_force_config(cfg))
    try:
        flags = (1 if exclusive else 0) | (2 if reverse else 0)
        check_status(L.scan_flat(xin.data_ptr(), out.data_ptr(), a.size, DT[a.dtype], flags, stream()),
                     "scan_flat")
    finally:
        if cfg is not None:
            L.scan_force_config(-1)
    torch.cuda.synchronize()
    return from_dev(out, a.dtype)


def segmented(a: np.ndarray, offsets: np.ndarray, exclusive=False, reverse=False, cfg=None):
    L = lib()
    x = to_dev(a)
    out = torch.empty_like(x)
    off = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).cuda()
    if cfg is not None:
        check_status(L.scan_force_config(cfg))
    try:
        flags = (1 if exclusive else 0) | (2 if reverse else 0)
        check_status(L.scan_segmented_batch(x.data_ptr(), out.data_ptr(), off.data_ptr(),
                                            off.numel() - 1, a.size, DT[a.dtype], flags, stream()),
                     "scan_segmented_batch")
    finally:
        if cfg is not None:
            L.scan_force_config(-1)
    torch.cuda.synchronize()
    return from_dev(out, a.dtype)


def configs():
    import paper_2312_14874_amd as m
    return [m.config_info(c) for c in range(m.num_configs())]


def f32_bad(got: np.ndarray, ref: np.ndarray, abs_sums: np.ndarray, exp: int = -20) -> np.ndarray:
    """Indices where a float result fails the acceptance rule against the
    float64 oracle: where ref is finite, got must be finite and within
    2^exp * running sum of |a| of it (a NaN or infinite output fails: the
    test is written so that a NaN compares as out of bound); where ref is
    NaN, got must be NaN; where ref is +-inf, got must be the same infinity.
    -0.0 and +0.0 compare equal."""
    g = np.asarray(got).astype(np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref)
    tol = np.ldexp(np.asarray(abs_sums, dtype=np.float64), exp)
    with np.errstate(invalid="ignore"):
        ok_fin = np.abs(g - ref) <= tol
        ok_nf = np.where(np.isnan(ref), np.isnan(g), g == ref)
    return np.nonzero(np.where(fin, ~ok_fin, ~ok_nf))[0]


def assert_f32_close(got: np.ndarray, ref: np.ndarray, abs_sums: np.ndarray, what=""):
    """float32 acceptance: |got - ref| <= 2^-20 * running sum of |a| (ref: float64
    oracle), non-finite values matched by class (see f32_bad)."""
    bad = f32_bad(got, ref, abs_sums)
    if bad.size:
        i = int(bad[0])
        raise AssertionError("%s: %d elements out of bound, first %d: got %r ref %r tol %r" % (
            what, bad.size, i, float(got[i]), float(ref[i]), float(np.ldexp(abs_sums[i], -20))))


def first_mismatch(got: np.ndarray, want: np.ndarray) -> str:
    bad = np.nonzero(got != want)[0]
    if bad.size == 0:
        return ""
    i = int(bad[0])
    return "%d mismatches, first at %d: got %r want %r" % (bad.size, i, got[i], want[i])
