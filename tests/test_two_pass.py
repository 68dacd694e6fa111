"""The two-pass comparison scans (Section 2.1 algorithms, optionally over the
cache-sized partitions of Section 2.2) against the oracle: the same results
contract as the single-pass scan (bit-exact for integers, the float32 bound),
for both methods, inclusive and exclusive, ragged sizes, partitions that do
and do not divide the array, in place and misaligned buffers."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import DT, assert_f32_close, check_status, first_mismatch, from_dev, lib, stream, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TILE = 16384
METHODS = [0, 1]   # prefix + increment, accumulate + prefix


def two_pass(a, method, exclusive=False, partition=0, inplace=False, misalign=0):
    L = lib()
    x = to_dev(a, pad=misalign + 4)
    xin = x[misalign + 4:]
    out = xin if inplace else torch.empty(a.size + misalign + 4, dtype=x.dtype, device="cuda")[misalign + 4:]
    check_status(L.scan_two_pass(xin.data_ptr(), out.data_ptr(), a.size, DT[a.dtype], 1 if exclusive else 0,
                                 method, partition, stream()), "scan_two_pass")
    torch.cuda.synchronize()
    return from_dev(out, a.dtype)


SIZES = [1, 7, TILE - 1, TILE, TILE + 1, 5 * TILE + 4321, 1 << 20]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("n", SIZES)
def test_int_sizes(method, n):
    a = workloads.full_u32(n, seed=2100 + n % 97)
    for ex in (False, True):
        got = two_pass(a, method, exclusive=ex)
        assert not first_mismatch(got, oracle.scan_int(a, exclusive=ex)), (method, n, ex)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("partition", [TILE, 3 * TILE + 5, 1 << 18])
def test_int_partitions(method, partition):
    n = 23 * TILE + 999                       # partitions do not divide the array
    a = workloads.full_u32(n, seed=2201)
    for ex in (False, True):
        got = two_pass(a, method, exclusive=ex, partition=partition)
        assert not first_mismatch(got, oracle.scan_int(a, exclusive=ex)), (method, partition, ex)


@pytest.mark.parametrize("method", METHODS)
def test_in_place_and_misaligned(method):
    a = workloads.uniform_i32(9 * TILE + 77, seed=2301)
    want = oracle.scan_int(a)
    assert not first_mismatch(two_pass(a, method, inplace=True), want)
    for mis in (1, 2, 3):
        assert not first_mismatch(two_pass(a, method, misalign=mis, partition=2 * TILE), want), mis


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("partition", [0, 4 * TILE])
def test_f32(method, partition):
    a = workloads.normal_f32(37 * TILE + 1234, seed=2401)
    for ex in (False, True):
        got = two_pass(a, method, exclusive=ex, partition=partition)
        ref, ab = oracle.scan_f32(a, exclusive=ex)
        assert_f32_close(got, ref, ab, "two-pass f32 method %d partition %d ex %d" % (method, partition, ex))


@pytest.mark.parametrize("method", METHODS)
def test_full_size_u32(method):
    """The single-pass benchmark workload (n = 2^28 full-range uint32), whole
    array and 2^24-element partitions, every element."""
    a = workloads.full_u32(1 << 28)
    want = oracle.scan_int(a)
    for part in (0, 1 << 24):
        assert not first_mismatch(two_pass(a, method, partition=part), want), part


def test_repeatable_f32():
    a = workloads.normal_f32(11 * TILE + 5, seed=2501)
    r1 = two_pass(a, 1, partition=3 * TILE)
    r2 = two_pass(a, 1, partition=3 * TILE)
    assert np.array_equal(r1.view(np.uint32), r2.view(np.uint32))
