"""The allocation-free flat scan (scan_flat_noalloc) against scan_flat, through
the C ABI: the same results on two calls in a row, the second with a smaller
input, for integer, float32, exclusive, reverse and max scans; integers
bit-exact, float32 bit-identical to scan_flat (the same configuration and
summation order) and within 2^-20 * sum|a| of the oracle.  Also: a forced
timeout of its bounded waits is reported by scan_check_device_error and
cleared, and the next calls are exact again."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_f32_close, check_status, from_dev, lib, stream, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

I32, U32, F32 = 0, 1, 2
EXCL, REV, OP_MAX = 0x1, 0x2, 0x4
TIMEOUT = 7


def _inputs(n, dt, seed):
    if dt == F32:
        return workloads.normal_f32(n, seed=seed)
    g = np.random.default_rng(seed)
    a = g.integers(0, 1 << 32, size=n, dtype=np.uint32)
    return a.view(np.int32) if dt == I32 else a


def _both(a, dt, flags, inplace=False):
    """(noalloc result, scan_flat result) on copies of a."""
    L = lib()
    res = []
    for entry in (L.scan_flat_noalloc, L.scan_flat):
        x = to_dev(a)
        y = x if inplace else torch.empty_like(x)
        print("%s n=%d dtype=%d flags=%#x inplace=%s" % (entry.__name__, a.size, dt, flags, inplace), flush=True)
        check_status(entry(x.data_ptr(), y.data_ptr(), a.size, dt, flags, stream()), entry.__name__)
        torch.cuda.synchronize()
        res.append(from_dev(y, a.dtype))
    assert L.scan_check_device_error(stream()) == 0
    return res


def _check(a, dt, flags, got, want):
    if dt == F32:
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), "float32 bits differ from scan_flat"
        ref, ab = oracle.scan_f32(a, exclusive=bool(flags & EXCL), reverse=bool(flags & REV))
        assert_f32_close(got, ref, ab)
    else:
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, "first mismatch at %d of %d" % (bad[0], a.size)
        if not flags & OP_MAX:
            ref = oracle.scan_int(a, exclusive=bool(flags & EXCL), reverse=bool(flags & REV))
            assert np.array_equal(got.view(np.uint32), np.asarray(ref).view(np.uint32))


# (dtype, flags, first n, second n): the first call spans many tiles with a
# ragged tail, the second is smaller (and lands in another tuning bucket)
CASES = [
    (U32, 0, (1 << 28) + 1001, 3 * 98304 + 17),
    (I32, EXCL, (1 << 24) + 77, 5000),
    (F32, 0, (1 << 24) + 3, 1 << 20),
    (F32, EXCL | REV, 3 * 98304 + 5, 70000),
    (U32, REV, (1 << 22) + 9, 4096 * 3 + 1),
    (I32, OP_MAX, (1 << 21) + 1, 255),
]


@pytest.mark.parametrize("dt,flags,n1,n2", CASES)
def test_noalloc_equals_scan_flat_on_two_calls(dt, flags, n1, n2):
    for k, n in enumerate((n1, n2)):
        a = _inputs(n, dt, seed=7300 + 10 * k + dt)
        got, want = _both(a, dt, flags)
        _check(a, dt, flags, got, want)


def test_noalloc_in_place_and_misaligned():
    L = lib()
    a = _inputs((1 << 20) + 33, U32, seed=7390)
    got, want = _both(a, U32, 0, inplace=True)
    _check(a, U32, 0, got, want)
    # a buffer 4 bytes past a 16-byte boundary takes the dword-access kernels
    n = 200001
    a = _inputs(n, U32, seed=7391)
    x = to_dev(a, pad=1)
    y = torch.empty(n + 1, dtype=x.dtype, device="cuda")
    check_status(L.scan_flat_noalloc(x[1:].data_ptr(), y[1:].data_ptr(), n, U32, 0, stream()), "noalloc")
    torch.cuda.synchronize()
    ref = oracle.scan_int(a)
    assert np.array_equal(from_dev(y[1:], np.uint32), np.asarray(ref).view(np.uint32))


SMALL_TILES = 11      # 256 threads x 16 items, one tile per workgroup from the counter


def test_noalloc_timeout_is_reported_and_cleared():
    L = lib()
    import paper_2312_14874_amd as scan
    info = scan.config_info(SMALL_TILES)
    assert info["tile"] == 4096 and info["mode"] == 0, info
    a = _inputs(1 << 24, U32, seed=7395)
    x = to_dev(a)
    y = torch.empty_like(x)
    seen = []
    check_status(L.scan_set_spin_limit(1))
    check_status(L.scan_force_config(SMALL_TILES))
    try:
        for _ in range(4):
            check_status(L.scan_flat_noalloc(x.data_ptr(), y.data_ptr(), a.size, U32, 0, stream()), "noalloc")
            seen.append(L.scan_check_device_error(stream()))
    finally:
        check_status(L.scan_set_spin_limit(0))
        check_status(L.scan_force_config(-1))
    assert all(s in (0, TIMEOUT) for s in seen), seen
    assert TIMEOUT in seen, "no wait gave up with a spin limit of one poll: %r" % seen
    assert L.scan_check_device_error(stream()) == 0
    for n in (a.size, 100003):
        check_status(L.scan_flat_noalloc(x.data_ptr(), y.data_ptr(), n, U32, 0, stream()), "noalloc")
        torch.cuda.synchronize()
        ref = oracle.scan_int(a[:n])
        assert np.array_equal(from_dev(y[:n], np.uint32), np.asarray(ref).view(np.uint32))
    assert L.scan_check_device_error(stream()) == 0
