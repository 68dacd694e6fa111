"""Batched segmented scans (one launch) against the oracle's per-segment
scans, and against per-segment launches of the flat scan."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_f32_close, configs, first_mismatch, segmented

pytestmark = pytest.mark.gpu

try:
    from paper_2312_14874_amd import num_configs
    NUM_CONFIGS = num_configs()
except ImportError:   # library not built: the GPU tests cannot run anyway
    NUM_CONFIGS = 1


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_int_random_offsets_every_config(cfg):
    g = np.random.default_rng(100 + cfg)
    tile = configs()[cfg]["tile"]
    for n, S in ((1, 1), (300, 7), (tile + 5, 40), (9 * tile + 17, 3), (40 * tile + 1, 900)):
        a = workloads.full_u32(n, seed=n + cfg)
        off = workloads.random_offsets(g, n, S)
        for ex in (False, True):
            for rev in (False, True):
                got = segmented(a, off, exclusive=ex, reverse=rev, cfg=cfg)
                want = oracle.segmented_int(a, off, exclusive=ex, reverse=rev)
                msg = first_mismatch(got, want)
                assert not msg, "cfg %d n %d S %d ex %d rev %d: %s" % (cfg, n, S, ex, rev, msg)


# starts on the boundaries the kernels treat apart -- a lane's 4-group, a
# 256-element chunk, a wave's span, a tile -- and one element either side;
# integer sums take the flat scan plus a subtraction per start, so these are
# the places where a start's prefix is read across lanes, chunks and waves
@pytest.mark.parametrize("cfg", [0, 1, 5, 7, 20, 21, 22, 30, 35])
def test_int_starts_on_boundaries(cfg):
    c = configs()[cfg]
    tile, wspan = c["tile"], 64 * c["items"]
    n = 5 * tile + 3 * wspan + 777
    cuts = set()
    for unit in (4, 256, wspan, tile):
        step = max(1, (n // unit) // 9)
        for m in range(1, n // unit + 1, step):
            for d in (-1, 0, 1):
                if 0 < m * unit + d < n:
                    cuts.add(m * unit + d)
    off = np.array([0] + sorted(cuts) + [n], dtype=np.int64)
    a = workloads.full_u32(n, seed=cfg + 7)
    for ex in (False, True):
        for rev in (False, True):
            got = segmented(a, off, exclusive=ex, reverse=rev, cfg=cfg)
            want = oracle.segmented_int(a, off, exclusive=ex, reverse=rev)
            msg = first_mismatch(got, want)
            assert not msg, "cfg %d ex %d rev %d: %s" % (cfg, ex, rev, msg)


# clusters of very short segments (lengths 1-4, so a lane's 4-group and a
# 256-element chunk hold several starts, some in the same lane) between long
# ones: the integer correction walks every start of a chunk in order
@pytest.mark.parametrize("cfg", [0, 1, 2, 5, 20, 21, 22, 30, 35])
def test_int_dense_start_clusters(cfg):
    c = configs()[cfg]
    tile, wspan = c["tile"], 64 * c["items"]
    n = 3 * tile + 2 * wspan + 1234
    g = np.random.default_rng(500 + cfg)
    cuts = set()
    centres = [wspan - 3, wspan + 250, tile - 1, tile + wspan // 2, 2 * tile + 256 * 5 - 2, n - 60]
    centres += list(g.integers(1, n - 1, size=4))
    for c0 in centres:
        x = int(c0)
        for _ in range(40):
            if 0 < x < n:
                cuts.add(x)
            x += int(g.integers(1, 5))
    off = np.array([0] + sorted(cuts) + [n], dtype=np.int64)
    a = workloads.full_u32(n, seed=cfg + 11)
    for ex in (False, True):
        for rev in (False, True):
            got = segmented(a, off, exclusive=ex, reverse=rev, cfg=cfg)
            want = oracle.segmented_int(a, off, exclusive=ex, reverse=rev)
            msg = first_mismatch(got, want)
            assert not msg, "cfg %d ex %d rev %d: %s" % (cfg, ex, rev, msg)


@pytest.mark.parametrize("cfg", [0, 2, 6, 9])
def test_f32_segments(cfg):
    g = np.random.default_rng(cfg)
    tile = configs()[cfg]["tile"]
    n = 25 * tile + 333
    a = workloads.normal_f32(n, seed=cfg)
    off = workloads.random_offsets(g, n, 60)
    for ex in (False, True):
        for rev in (False, True):
            got = segmented(a, off, exclusive=ex, reverse=rev, cfg=cfg)
            ref, ab = oracle.segmented_f32(a, off, exclusive=ex, reverse=rev)
            assert_f32_close(got, ref, ab, "cfg %d ex %d rev %d" % (cfg, ex, rev))


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_f32_segments_exact_when_sums_representable(cfg):
    # integer-valued float32 in [-2, 2], n < 2^22: every partial sum is exact,
    # so the segmented float32 kernels must match the oracle bit for bit
    g = np.random.default_rng(900 + cfg)
    n = (1 << 22) - 5
    a = workloads.small_int_f32(n, seed=cfg)
    off = workloads.random_offsets(g, n, 500)
    for ex in (False, True):
        for rev in (False, True):
            got = segmented(a, off, exclusive=ex, reverse=rev, cfg=cfg)
            ref, _ = oracle.segmented_f32(a, off, exclusive=ex, reverse=rev, with_abs=False)
            assert np.array_equal(got.astype(np.float64), ref), "cfg %d ex %d rev %d: %s" % (
                cfg, ex, rev, first_mismatch(got.astype(np.float64), ref))


def test_special_segmentations():
    n = 100_003
    a = workloads.full_u32(n, seed=3)
    # one segment == flat scan
    for ex in (False, True):
        assert not first_mismatch(segmented(a, np.array([0, n]), exclusive=ex),
                                  oracle.scan_int(a, exclusive=ex))
    # all length-1 segments
    off = np.arange(n + 1, dtype=np.int64)
    assert not first_mismatch(segmented(a, off), a)
    assert not first_mismatch(segmented(a, off, exclusive=True), np.zeros(n, dtype=np.uint32))
    # many empty segments, including leading and trailing ones
    off = np.array([0, 0, 0, 10, 10, 5000, 5000, n, n, n], dtype=np.int64)
    for ex in (False, True):
        for rev in (False, True):
            assert not first_mismatch(segmented(a, off, exclusive=ex, reverse=rev),
                                      oracle.segmented_int(a, off, exclusive=ex, reverse=rev))
