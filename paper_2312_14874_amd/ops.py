"""torch-facing wrappers: validate tensors, then call the C ABI.

torch supplies device memory and the stream (torch.cuda.current_stream());
every step of the scan runs in the HIP kernels of libmi355scan.so.
"""
from __future__ import annotations

import ctypes

import torch

from ._lib import (SCAN_EXCLUSIVE, SCAN_F32, SCAN_I32, SCAN_I64, SCAN_PRED_GREATER, SCAN_PRED_NONZERO,
                   SCAN_F64, SCAN_REVERSE, SCAN_TWO_PASS_ACCUMULATE_PREFIX, SCAN_TWO_PASS_PREFIX_INCREMENT,
                   SCAN_U32, SCAN_U64, check, lib)

_DTYPES = {torch.int32: SCAN_I32, torch.float32: SCAN_F32}
if hasattr(torch, "uint32"):
    _DTYPES[torch.uint32] = SCAN_U32
# 64-bit elements: +-scans of cumsum only (the library refuses the rest)
_DTYPES[torch.int64] = SCAN_I64
_DTYPES[torch.float64] = SCAN_F64
if hasattr(torch, "uint64"):
    _DTYPES[torch.uint64] = SCAN_U64


def _stream(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


# operator field of the flags (bits 2-3): + (default), max, min, xor
OPERATORS = {"sum": 0x0, "max": 0x4, "min": 0x8, "xor": 0xC}


def _flags(exclusive: bool, reverse: bool, op: str = "sum") -> int:
    if op not in OPERATORS:
        raise ValueError("op must be one of %s" % sorted(OPERATORS))
    return (SCAN_EXCLUSIVE if exclusive else 0) | (SCAN_REVERSE if reverse else 0) | OPERATORS[op]


def _check_tensor(x: torch.Tensor, name: str) -> int:
    if not isinstance(x, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not x.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if x.dtype not in _DTYPES:
        raise TypeError("%s: unsupported dtype %s (int32, uint32, float32, int64, uint64, float64)" % (name, x.dtype))
    if not x.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return _DTYPES[x.dtype]


def _out_like(x: torch.Tensor, out):
    if out is None:
        return torch.empty_like(x)
    if out.dtype != x.dtype or out.numel() != x.numel() or out.device != x.device or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor with the input's dtype, size and device")
    return out


def _check_offsets(offsets: torch.Tensor, x: torch.Tensor) -> int:
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or not offsets.is_contiguous():
        raise TypeError("offsets must be a contiguous 1-D int64 tensor")
    if offsets.device != x.device:
        raise ValueError("offsets must be on the input's device")
    if offsets.numel() < 1:
        raise ValueError("offsets needs num_segments + 1 entries")
    return offsets.numel() - 1


def cumsum(x: torch.Tensor, exclusive: bool = False, reverse: bool = False, out=None,
           op: str = "sum") -> torch.Tensor:
    """Scan of a contiguous int32 / uint32 / float32 GPU tensor (flattened).

    op: "sum" (any dtype), or "max" / "min" / "xor" for int32 (signed) and
    uint32.  out may be x itself (in place).  int64 / uint64 / float64
    tensors take +-scans (exclusive, reverse or not; integers wrap modulo
    2^64) and must start on a 16-byte boundary."""
    dt = _check_tensor(x, "x")
    out = _out_like(x, out)
    with torch.cuda.device(x.device):
        check(lib.scan_flat(x.data_ptr(), out.data_ptr(), x.numel(), dt,
                            _flags(exclusive, reverse, op), _stream(x.device)), "scan_flat")
    return out


def exclusive_cumsum(x: torch.Tensor, out=None) -> torch.Tensor:
    return cumsum(x, exclusive=True, out=out)


def segmented_scan(x: torch.Tensor, offsets: torch.Tensor, exclusive: bool = False,
                   reverse: bool = False, out=None, op: str = "sum") -> torch.Tensor:
    """Independent scans of the segments x[offsets[s]:offsets[s+1]] in one launch
    (op as for cumsum)."""
    dt = _check_tensor(x, "x")
    S = _check_offsets(offsets, x)
    out = _out_like(x, out)
    with torch.cuda.device(x.device):
        check(lib.scan_segmented_batch(x.data_ptr(), out.data_ptr(), offsets.data_ptr(), S,
                                       x.numel(), dt, _flags(exclusive, reverse, op),
                                       _stream(x.device)), "scan_segmented_batch")
    return out


def segmented_scan_looped(x: torch.Tensor, host_offsets, exclusive: bool = False,
                          reverse: bool = False, out=None) -> torch.Tensor:
    """Comparator: one flat-scan launch per segment (host_offsets on the CPU)."""
    import numpy as np
    dt = _check_tensor(x, "x")
    off = np.ascontiguousarray(np.asarray(host_offsets, dtype=np.int64))
    out = _out_like(x, out)
    with torch.cuda.device(x.device):
        check(lib.scan_segmented_looped(x.data_ptr(), out.data_ptr(), off.ctypes.data, off.size - 1,
                                        dt, _flags(exclusive, reverse), _stream(x.device)),
              "scan_segmented_looped")
    return out


PREDICATES = {"nonzero": SCAN_PRED_NONZERO, "greater": SCAN_PRED_GREATER}


def _select_args(x, out, count, predicate, threshold):
    if predicate not in PREDICATES:
        raise ValueError("predicate must be one of %s" % sorted(PREDICATES))
    dt = _check_tensor(x, "x")
    out = _out_like(x, out)
    if count.dtype != torch.int64 or count.numel() != 1 or count.device != x.device:
        raise ValueError("count must be a one-element int64 tensor on x's device")
    thr = torch.tensor([threshold], dtype=x.dtype).view(torch.int32).item() & 0xFFFFFFFF
    return dt, out, thr


def compact_into(x: torch.Tensor, out: torch.Tensor, count: torch.Tensor, predicate: str = "nonzero",
                 threshold=0) -> None:
    """Asynchronous stream compaction: out[:count] receives, in order, the
    elements of x the predicate keeps ("nonzero", or "greater": x > threshold
    in x's type); count is a one-element int64 GPU tensor."""
    dt, out, thr = _select_args(x, out, count, predicate, threshold)
    with torch.cuda.device(x.device):
        check(lib.scan_compact(x.data_ptr(), out.data_ptr(), x.numel(), dt, PREDICATES[predicate], thr,
                               count.data_ptr(), _stream(x.device)), "scan_compact")


def partition_into(x: torch.Tensor, out: torch.Tensor, count: torch.Tensor, predicate: str = "nonzero",
                   threshold=0) -> None:
    """Asynchronous two-way partition: out[:count] receives the elements of x
    the predicate keeps, in order, and out[count:] the others in reverse
    order; out must not overlap x."""
    dt, out, thr = _select_args(x, out, count, predicate, threshold)
    with torch.cuda.device(x.device):
        check(lib.scan_partition(x.data_ptr(), out.data_ptr(), x.numel(), dt, PREDICATES[predicate], thr,
                                 count.data_ptr(), _stream(x.device)), "scan_partition")


def partition(x: torch.Tensor, predicate: str = "nonzero", threshold=0):
    """(out, k): the kept elements of x in out[:k] in order, the others in
    out[k:] in reverse order (synchronises to read k)."""
    out = torch.empty_like(x)
    count = torch.empty(1, dtype=torch.int64, device=x.device)
    partition_into(x, out, count, predicate, threshold)
    return out, int(count.item())


def compact(x: torch.Tensor, predicate: str = "nonzero", threshold=0) -> torch.Tensor:
    """The elements of x the predicate keeps, in order (synchronises to read
    the count)."""
    out = torch.empty_like(x)
    count = torch.empty(1, dtype=torch.int64, device=x.device)
    compact_into(x, out, count, predicate, threshold)
    return out[:int(count.item())]


TWO_PASS_METHODS = {"prefix_increment": SCAN_TWO_PASS_PREFIX_INCREMENT,
                    "accumulate_prefix": SCAN_TWO_PASS_ACCUMULATE_PREFIX}


def two_pass_cumsum(x: torch.Tensor, method: str = "accumulate_prefix", exclusive: bool = False,
                    partition: int = 0, out=None) -> torch.Tensor:
    """Comparison path: the same scan by one of the paper's two-pass algorithms
    ("prefix_increment": scan then add offsets, 16 B/element of HBM traffic;
    "accumulate_prefix": sum then scan with offsets, 12 B/element), over
    partitions of `partition` elements (0 = one partition)."""
    if method not in TWO_PASS_METHODS:
        raise ValueError("method must be one of %s" % sorted(TWO_PASS_METHODS))
    dt = _check_tensor(x, "x")
    out = _out_like(x, out)
    with torch.cuda.device(x.device):
        check(lib.scan_two_pass(x.data_ptr(), out.data_ptr(), x.numel(), dt, _flags(exclusive, False),
                                TWO_PASS_METHODS[method], int(partition), _stream(x.device)),
              "scan_two_pass")
    return out


def cumsum_backward(grad: torch.Tensor, offsets=None, out=None) -> torch.Tensor:
    """Gradient of an inclusive cumsum: per-segment suffix sums of grad
    (float32; float64 without offsets)."""
    dt = _check_tensor(grad, "grad")
    if dt == SCAN_F64 and offsets is None:
        return cumsum(grad, reverse=True, out=out)
    if dt != SCAN_F32:
        raise TypeError("cumsum_backward takes float32 (float64 without offsets)")
    out = _out_like(grad, out)
    with torch.cuda.device(grad.device):
        if offsets is None:
            check(lib.scan_f32_backward(grad.data_ptr(), out.data_ptr(), grad.numel(), None, 0,
                                        _stream(grad.device)), "scan_f32_backward")
        else:
            S = _check_offsets(offsets, grad)
            check(lib.scan_f32_backward(grad.data_ptr(), out.data_ptr(), grad.numel(),
                                        offsets.data_ptr(), S, _stream(grad.device)),
                  "scan_f32_backward")
    return out


class CumsumFn(torch.autograd.Function):
    """Differentiable inclusive cumsum: float32 over a flat tensor or over the
    ragged rows given by CSR offsets, float64 over a flat tensor.  The
    backward is the reverse (suffix) scan; nothing but the offsets is saved,
    because the map is linear."""

    @staticmethod
    def forward(ctx, x, offsets=None):
        if x.dtype != torch.float32 and not (x.dtype == torch.float64 and offsets is None):
            raise TypeError("CumsumFn takes float32 (float64 without offsets)")
        xc = x.contiguous()
        y = cumsum(xc) if offsets is None else segmented_scan(xc, offsets)
        ctx.offsets = offsets
        return y

    @staticmethod
    def backward(ctx, gy):
        return cumsum_backward(gy.contiguous(), ctx.offsets), None


def cumsum_autograd(x: torch.Tensor, offsets=None) -> torch.Tensor:
    return CumsumFn.apply(x, offsets)


class SegmentedScanGraph:
    """A batched segmented scan captured once into a hipGraph and replayed.

    The tensors are bound at construction; change their contents, not their
    storage, between replays."""

    def __init__(self, x: torch.Tensor, out: torch.Tensor, offsets: torch.Tensor,
                 exclusive: bool = False, reverse: bool = False):
        dt = _check_tensor(x, "x")
        S = _check_offsets(offsets, x)
        _out_like(x, out)
        self._keep = (x, out, offsets)
        self.device = x.device
        h = ctypes.c_void_p()
        with torch.cuda.device(x.device):
            check(lib.scan_segmented_graph_create(x.data_ptr(), out.data_ptr(), offsets.data_ptr(), S,
                                                  x.numel(), dt, _flags(exclusive, reverse),
                                                  _stream(x.device), ctypes.byref(h)),
                  "scan_segmented_graph_create")
        self._h = h

    def launch(self):
        with torch.cuda.device(self.device):
            check(lib.scan_graph_launch(self._h, _stream(self.device)), "scan_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            with torch.cuda.device(self.device):
                lib.scan_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LoopedScanGraph(SegmentedScanGraph):
    """Comparator: one flat-scan launch per segment, captured into one graph."""

    def __init__(self, x: torch.Tensor, out: torch.Tensor, host_offsets,
                 exclusive: bool = False, reverse: bool = False):
        import numpy as np
        dt = _check_tensor(x, "x")
        _out_like(x, out)
        off = np.ascontiguousarray(np.asarray(host_offsets, dtype=np.int64))
        self._keep = (x, out, off)
        self.device = x.device
        h = ctypes.c_void_p()
        with torch.cuda.device(x.device):
            check(lib.scan_looped_graph_create(x.data_ptr(), out.data_ptr(), off.ctypes.data,
                                               off.size - 1, dt, _flags(exclusive, reverse),
                                               _stream(x.device), ctypes.byref(h)),
                  "scan_looped_graph_create")
        self._h = h


def num_configs() -> int:
    return lib.scan_num_configs()


def config_info(cfg: int) -> dict:
    b, i, nt, p, pc, sg = (ctypes.c_int32() for _ in range(6))
    check(lib.scan_config_info(cfg, ctypes.byref(b), ctypes.byref(i), ctypes.byref(nt), ctypes.byref(p),
                               ctypes.byref(pc), ctypes.byref(sg)))
    return {"config": cfg, "block": b.value, "items": i.value, "nontemporal": nt.value,
            "mode": p.value, "per_cu": pc.value, "cu_pct": sg.value, "tile": b.value * i.value}


def force_config(cfg: int = -1) -> None:
    check(lib.scan_force_config(cfg), "scan_force_config")


def selected_config(dtype: torch.dtype, n: int, segmented: bool = False, flags: int = 0) -> int:
    return lib.scan_selected_config(_DTYPES[dtype], flags, int(segmented), n)


def autotune(x: torch.Tensor, out: torch.Tensor, offsets=None, exclusive: bool = False,
             reverse: bool = False, reps: int = 5) -> int:
    dt = _check_tensor(x, "x")
    best = ctypes.c_int32(-1)
    off_ptr, S = None, 0
    if offsets is not None:
        S = _check_offsets(offsets, x)
        off_ptr = offsets.data_ptr()
    with torch.cuda.device(x.device):
        check(lib.scan_autotune(x.data_ptr(), out.data_ptr(), x.numel(), off_ptr, S, dt,
                                _flags(exclusive, reverse), reps, _stream(x.device),
                                ctypes.byref(best)), "scan_autotune")
    return best.value


def tune_save(path: str) -> None:
    check(lib.scan_tune_save(path.encode()), "scan_tune_save")


def tune_load(path: str) -> None:
    check(lib.scan_tune_load(path.encode()), "scan_tune_load")


def reserve(max_n: int, device=None) -> None:
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        check(lib.scan_reserve(max_n, _stream(dev)), "scan_reserve")


def set_spin_limit(limit: int) -> None:
    check(lib.scan_set_spin_limit(limit), "scan_set_spin_limit")


def check_device_error(device=None) -> int:
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    with torch.cuda.device(dev):
        return lib.scan_check_device_error(_stream(dev))
