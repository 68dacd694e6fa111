"""Parity at the full benchmark sizes, in the launch configuration the
library selects by default (the one bench.py times), against the sequential
oracle on every element:

  * uint32 full-range inclusive scan, n = 2^28 (the headline workload),
    out of place and in place, and n = 2^30;
  * float32 normal(0, 1), n = 2^28, inclusive and exclusive, within
    2^-20 * sum |a_j|;
  * the batched exclusive segmented scan over S = 4096 log-uniform segments
    (n = 328,685,534 Poisson(8) int32 values).

Host memory: about 12 GB at n = 2^30; device memory 8 GB."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_f32_close, first_mismatch, flat, segmented

pytestmark = pytest.mark.gpu


def test_u32_n2p28_bench_workload():
    a = workloads.full_u32(1 << 28)
    want = oracle.scan_int(a)
    got = flat(a)
    assert not first_mismatch(got, want)
    # in place, exclusive
    got = flat(a, exclusive=True, inplace=True)
    assert not first_mismatch(got, oracle.scan_int(a, exclusive=True))


def test_u32_n2p30():
    a = workloads.full_u32(1 << 30, seed=1012)
    got = flat(a)
    want = oracle.scan_int(a)
    assert not first_mismatch(got, want)


def test_f32_n2p28():
    a = workloads.normal_f32(1 << 28)
    for ex in (False, True):
        got = flat(a, exclusive=ex)
        ref, ab = oracle.scan_f32(a, exclusive=ex)
        assert_f32_close(got, ref, ab, "f32 n=2^28 ex %d" % ex)
        del ref, ab, got


def test_segmented_s4096_bench_workload():
    vals, off = workloads.segments()
    got = segmented(vals, off, exclusive=True)
    want = oracle.segmented_int(vals, off, exclusive=True)
    assert not first_mismatch(got, want)
