"""Flat scans on the GPU against the sequential oracle.

Integers (int32 / uint32, wrapping) must match bit for bit; float32 must stay
within 2^-20 * sum_{j<=i} |a_j| of the float64 oracle, and be bit-exact where
every partial sum is representable.  Sizes span several tiles of every
configuration plus a ragged tail."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_f32_close, configs, first_mismatch, flat

pytestmark = pytest.mark.gpu

try:
    from paper_2312_14874_amd import num_configs
    NUM_CONFIGS = num_configs()
except ImportError:   # library not built: the GPU tests cannot run anyway
    NUM_CONFIGS = 1


def _sizes(tile):
    return [1, 63, 64, 65, 255, 257, tile - 1, tile, tile + 1, 3 * tile + 123, 131 * tile + 4099]


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_u32_every_config(cfg):
    info = configs()[cfg]
    for n in _sizes(info["tile"]):
        a = workloads.full_u32(n, seed=n + cfg)
        for ex in (False, True):
            for rev in (False, True):
                got = flat(a, exclusive=ex, reverse=rev, cfg=cfg)
                want = oracle.scan_int(a, exclusive=ex, reverse=rev)
                msg = first_mismatch(got, want)
                assert not msg, "cfg %d n %d ex %d rev %d: %s" % (cfg, n, ex, rev, msg)


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_f32_every_config(cfg):
    info = configs()[cfg]
    for n in (1, 257, info["tile"] + 1, 37 * info["tile"] + 999):
        a = workloads.normal_f32(n, seed=7 * n + cfg)
        for ex in (False, True):
            for rev in (False, True):
                got = flat(a, exclusive=ex, reverse=rev, cfg=cfg)
                ref, ab = oracle.scan_f32(a, exclusive=ex, reverse=rev)
                assert_f32_close(got, ref, ab, "cfg %d n %d ex %d rev %d" % (cfg, n, ex, rev))
                if ex:
                    first = -1 if rev else 0
                    assert got[first] == 0.0


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_f32_exact_when_sums_representable(cfg):
    # integers in [-2, 2], n <= 2^22: every partial sum fits in 24 bits, so
    # every association gives the same bits and a dropped or repeated
    # element anywhere shows (the 2^-20 bound alone would miss one near the
    # end of a long array)
    for n in (5000, 1 << 20, (1 << 22) - 3):
        a = workloads.small_int_f32(n, seed=n)
        for ex in (False, True):
            for rev in (False, True):
                got = flat(a, exclusive=ex, reverse=rev, cfg=cfg)
                ref, _ = oracle.scan_f32(a, exclusive=ex, reverse=rev, with_abs=False)
                assert np.array_equal(got.astype(np.float64), ref), first_mismatch(got.astype(np.float64), ref)


def test_small_i32_workload_inclusive_and_exclusive():
    a = workloads.uniform_i32(1 << 20)
    for ex in (False, True):
        got = flat(a, exclusive=ex)
        want = oracle.scan_int(a, exclusive=ex)
        assert got.dtype == np.int32
        assert not first_mismatch(got, want)


@pytest.mark.parametrize("misalign", [1, 2, 3])
def test_misaligned_pointers(misalign):
    for n in (1000, 70_001):
        a = workloads.full_u32(n, seed=misalign)
        for ex in (False, True):
            got = flat(a, exclusive=ex, misalign=misalign)
            assert not first_mismatch(got, oracle.scan_int(a, exclusive=ex))
        f = workloads.normal_f32(n, seed=misalign)
        ref, ab = oracle.scan_f32(f)
        assert_f32_close(flat(f, misalign=misalign), ref, ab, "misaligned f32")


@pytest.mark.parametrize("rev", [False, True])
def test_in_place(rev):
    for n in (9, 100_000, 3_000_001):
        a = workloads.full_u32(n, seed=n)
        for ex in (False, True):
            got = flat(a, exclusive=ex, reverse=rev, inplace=True)
            assert not first_mismatch(got, oracle.scan_int(a, exclusive=ex, reverse=rev))


def test_closed_forms_on_device():
    n = 5_000_011
    ones = np.ones(n, dtype=np.int32)
    assert np.array_equal(flat(ones), np.arange(1, n + 1, dtype=np.int64).astype(np.int32))
    assert np.array_equal(flat(ones, exclusive=True), np.arange(n, dtype=np.int64).astype(np.int32))
    assert np.array_equal(flat(ones, reverse=True), np.arange(n, 0, -1, dtype=np.int64).astype(np.int32))


def test_f32_deterministic_run_to_run():
    a = workloads.normal_f32((1 << 22) + 77, seed=5)
    r0 = flat(a)
    for _ in range(5):
        assert np.array_equal(flat(a).view(np.uint32), r0.view(np.uint32))
