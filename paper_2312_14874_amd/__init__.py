"""mi355scan: single-pass prefix sums for AMD Instinct MI355X (gfx950).

A GPU counterpart of the scan studied in Zhang, Wang and Ross, "Parallel
Prefix Sum with SIMD" (ADMS 2020): each element is read from HBM once and
written once.  The kernels and the C ABI live in libmi355scan.so
(include/mi355scan.h); this package marshals torch tensors into it.
"""
from ._lib import (SCAN_EXCLUSIVE, SCAN_F32, SCAN_I32, SCAN_REVERSE, SCAN_U32,
                   LIB_PATH, ScanError, check, lib)
from .ops import (CumsumFn, LoopedScanGraph, SegmentedScanGraph, autotune,
                  check_device_error, config_info, cumsum, cumsum_autograd,
                  cumsum_backward, exclusive_cumsum, force_config, num_configs,
                  reserve, segmented_scan, segmented_scan_looped,
                  selected_config, set_spin_limit, tune_load, tune_save, two_pass_cumsum,
                  compact, compact_into, partition, partition_into)

__all__ = [
    "SCAN_EXCLUSIVE", "SCAN_F32", "SCAN_I32", "SCAN_REVERSE", "SCAN_U32", "LIB_PATH",
    "ScanError", "check", "lib", "CumsumFn", "LoopedScanGraph", "SegmentedScanGraph",
    "autotune", "check_device_error", "config_info", "cumsum", "cumsum_autograd",
    "cumsum_backward", "exclusive_cumsum", "force_config", "num_configs", "reserve",
    "segmented_scan", "segmented_scan_looped", "selected_config", "set_spin_limit",
    "tune_load", "tune_save", "two_pass_cumsum", "compact", "compact_into", "partition", "partition_into",
]
