"""Scans with the other associative operators of the Introduction's
definition (max, min, xor on int32 / uint32) against the oracle, bit-exact:
flat (several launch configurations, ragged tails, misaligned and in-place
buffers, the reverse forms the kernels take), segmented (empty segments
included), and the 2^28 workload size."""
import numpy as np
import pytest

import oracle
from gpu_util import DT, check_status, first_mismatch, from_dev, lib, stream, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OPF = {"max": 0x4, "min": 0x8, "xor": 0xC}
CONFIGS = [None, 4, 8, 11, 20, 22]


def walk(n, seed, dtype):
    """Values whose running max / min keep changing: a random walk with steps
    in [-40, 40] plus occasional spikes, spanning the signed and unsigned
    ranges (the int64 walk is wrapped into 32 bits)."""
    g = np.random.default_rng(seed)
    w = np.cumsum(g.integers(-40, 41, size=n)) + g.integers(-(1 << 31), 1 << 31)
    spikes = g.random(n) < 0.001
    w[spikes] += g.integers(-(1 << 30), 1 << 30, size=int(spikes.sum()))
    return (w % (1 << 32)).astype(np.uint32).view(dtype)


def run_flat(a, op, exclusive=False, reverse=False, cfg=None, misalign=0, inplace=False):
    L = lib()
    x = to_dev(a, pad=misalign + 4)
    xin = x[misalign + 4:]
    out = xin if inplace else torch.empty(a.size + misalign + 4, dtype=x.dtype, device="cuda")[misalign + 4:]
    flags = OPF[op] | (1 if exclusive else 0) | (2 if reverse else 0)
    if cfg is not None:
        check_status(L.scan_force_config(cfg))
    try:
        check_status(L.scan_flat(xin.data_ptr(), out.data_ptr(), a.size, DT[a.dtype], flags, stream()), "scan_flat")
    finally:
        if cfg is not None:
            L.scan_force_config(-1)
    torch.cuda.synchronize()
    return from_dev(out, a.dtype)


def run_seg(a, off, op, exclusive=False, reverse=False, cfg=None):
    L = lib()
    x = to_dev(a)
    out = torch.empty_like(x)
    o = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).cuda()
    flags = OPF[op] | (1 if exclusive else 0) | (2 if reverse else 0)
    if cfg is not None:
        check_status(L.scan_force_config(cfg))
    try:
        check_status(L.scan_segmented_batch(x.data_ptr(), out.data_ptr(), o.data_ptr(), o.numel() - 1, a.size,
                                            DT[a.dtype], flags, stream()), "scan_segmented_batch")
    finally:
        if cfg is not None:
            L.scan_force_config(-1)
    torch.cuda.synchronize()
    return from_dev(out, a.dtype)


def reverse_ok(op, dtype):
    return op == "xor" or (op == "max" and dtype == np.uint32)


@pytest.mark.parametrize("dtype", [np.int32, np.uint32])
@pytest.mark.parametrize("op", ["max", "min", "xor"])
@pytest.mark.parametrize("cfg", CONFIGS)
def test_flat(dtype, op, cfg):
    n = 3 * 98304 + 12345          # several tiles of every shape plus a ragged tail
    a = walk(n, 3000 + OPF[op] + (cfg or 0), dtype)
    for ex in (False, True):
        want = oracle.scan_op(a, op, exclusive=ex)
        got = run_flat(a, op, exclusive=ex, cfg=cfg)
        assert not first_mismatch(got, want), (op, np.dtype(dtype).name, cfg, ex)
    if reverse_ok(op, dtype):
        for ex in (False, True):
            want = oracle.scan_op(a, op, exclusive=ex, reverse=True)
            got = run_flat(a, op, exclusive=ex, reverse=True, cfg=cfg)
            assert not first_mismatch(got, want), (op, np.dtype(dtype).name, cfg, ex, "reverse")


# xor takes the integer sum's correction per segment start (it is its own
# inverse): runs of segments of length 1-4 put several starts in one lane
@pytest.mark.parametrize("cfg", [None, 5, 21, 35])
def test_segmented_xor_dense_starts(cfg):
    g = np.random.default_rng(3300 + (cfg or 0))
    lens = g.integers(1, 5, size=4000)
    lens[100:110] = 30000                            # long segments between the clusters
    lens[2000:2005] = 70000
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    a = walk(int(off[-1]), 3301, np.uint32)
    for ex in (False, True):
        for rev in (False, True):
            want = oracle.segmented_op(a, off, "xor", exclusive=ex, reverse=rev)
            got = run_seg(a, off, "xor", exclusive=ex, reverse=rev, cfg=cfg)
            assert not first_mismatch(got, want), (cfg, ex, rev)


@pytest.mark.parametrize("op", ["max", "min", "xor"])
@pytest.mark.parametrize("n", [1, 5, 4096, 65537, 1 << 20])
def test_sizes_misaligned_inplace(op, n):
    a = walk(n, 3100 + n % 101, np.int32)
    want = oracle.scan_op(a, op, exclusive=True)
    assert not first_mismatch(run_flat(a, op, exclusive=True, misalign=3), want), "misaligned"
    assert not first_mismatch(run_flat(a, op, exclusive=True, inplace=True), want), "in place"


@pytest.mark.parametrize("dtype", [np.int32, np.uint32])
@pytest.mark.parametrize("op", ["max", "min", "xor"])
@pytest.mark.parametrize("cfg", [None, 4, 20])
def test_segmented(dtype, op, cfg):
    g = np.random.default_rng(3200 + OPF[op])
    lens = g.integers(0, 40000, size=60)
    lens[::7] = 0                                    # empty segments
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    a = walk(int(off[-1]), 3201, dtype)
    for ex in (False, True):
        want = oracle.segmented_op(a, off, op, exclusive=ex)
        assert not first_mismatch(run_seg(a, off, op, exclusive=ex, cfg=cfg), want), (op, cfg, ex)
    if reverse_ok(op, dtype):
        want = oracle.segmented_op(a, off, op, exclusive=True, reverse=True)
        assert not first_mismatch(run_seg(a, off, op, exclusive=True, reverse=True, cfg=cfg), want), "reverse"


@pytest.mark.parametrize("op", ["max", "min", "xor"])
def test_full_size_int32(op):
    a = walk(1 << 28, 3300 + OPF[op], np.int32)
    want = oracle.scan_op(a, op, exclusive=True)
    assert not first_mismatch(run_flat(a, op, exclusive=True), want)
