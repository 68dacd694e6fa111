"""Failure handling of the bounded device-side waits, forced from the host:
with a spin limit of one poll, a tile that has to wait twice gives up, raises
the error word of its stream (or graph) and the kernel finishes normally
(results of that call invalid).  The next call on that stream, or the next
replay of that graph, reports SCAN_ERROR_TIMEOUT once and enqueues nothing;
scan_check_device_error reports it after synchronising; with the default
limit restored the next scans are exact again.  The 32-bit launches use the
one-tile-per-workgroup configuration with 4096-element tiles, whose thousands
of tiles start together, so some of them are sure to wait; every wait stays
bounded, so every kernel ends."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import check_status, first_mismatch, flat, lib, stream, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TIMEOUT = 7
SMALL_TILES = 11      # 256 threads x 16 items, one tile per workgroup from the counter


def _small_tile_config():
    import paper_2312_14874_amd as scan
    info = scan.config_info(SMALL_TILES)
    assert info["tile"] == 4096 and info["mode"] == 0, info
    return SMALL_TILES


def test_spin_limit_timeout_is_reported_and_cleared():
    L = lib()
    cfg = _small_tile_config()
    g = np.random.default_rng(7200)
    a32 = g.integers(0, 1 << 32, size=1 << 24, dtype=np.uint32)
    a64 = g.integers(0, 1 << 64, size=1 << 25, dtype=np.uint64)
    x32 = to_dev(a32)
    y32 = torch.empty_like(x32)
    x64 = torch.from_numpy(a64.view(np.int64)).cuda()
    y64 = torch.empty_like(x64)
    seen = []
    check_status(L.scan_set_spin_limit(1))
    check_status(L.scan_force_config(cfg))
    try:
        for _ in range(4):
            check_status(L.scan_flat(x32.data_ptr(), y32.data_ptr(), a32.size, 1, 0, stream()), "scan_flat")
            seen.append(L.scan_check_device_error(stream()))
            check_status(L.scan_flat(x64.data_ptr(), y64.data_ptr(), a64.size, 4, 0, stream()), "scan_flat u64")
            seen.append(L.scan_check_device_error(stream()))
    finally:
        check_status(L.scan_set_spin_limit(0))
        check_status(L.scan_force_config(-1))
    assert all(s in (0, TIMEOUT) for s in seen), seen
    assert TIMEOUT in seen, "no wait gave up with a spin limit of one poll: %r" % seen
    print("timeouts reported: %d of %d calls" % (seen.count(TIMEOUT), len(seen)))
    # each check cleared the word, and the workspace still works
    assert L.scan_check_device_error(stream()) == 0
    assert not first_mismatch(flat(a32), np.asarray(oracle.scan_int(a32)))
    check_status(L.scan_flat(x64.data_ptr(), y64.data_ptr(), a64.size, 4, 0, stream()), "scan_flat u64")
    torch.cuda.synchronize()
    assert not first_mismatch(y64.cpu().numpy().view(np.uint64), oracle.scan_int64(a64))
    assert L.scan_check_device_error(stream()) == 0


def test_timeout_surfaces_through_cumsum():
    import paper_2312_14874_amd as scan
    cfg = _small_tile_config()
    a = workloads.full_u32(1 << 24, seed=7300)
    x = to_dev(a)
    y = torch.empty_like(x)
    raised = None
    scan.set_spin_limit(1)
    scan.force_config(cfg)
    try:
        for _ in range(8):
            try:
                scan.cumsum(x, out=y)
                torch.cuda.synchronize()
            except scan.ScanError as e:
                raised = e
                break
    finally:
        scan.set_spin_limit(0)
        scan.force_config(-1)
    assert raised is not None, "no timeout reported through cumsum() in 8 launches"
    assert raised.status == TIMEOUT and "earlier call" in str(raised)
    # reported once: the next call runs, and is exact
    y.zero_()
    scan.cumsum(x, out=y)
    torch.cuda.synchronize()
    assert not first_mismatch(y.cpu().numpy().view(np.uint32), oracle.scan_int(a))
    assert scan.check_device_error() == 0


def test_timeout_surfaces_through_graph_replay():
    import paper_2312_14874_amd as scan
    L = lib()
    cfg = _small_tile_config()
    n = 1 << 24
    a = workloads.full_u32(n, seed=7400)
    off = workloads.random_offsets(np.random.default_rng(7400), n, 64)
    x = to_dev(a)
    y = torch.empty_like(x)
    offs = torch.from_numpy(off).cuda()
    scan.set_spin_limit(1)
    scan.force_config(cfg)
    try:
        g = scan.SegmentedScanGraph(x, y, offs)      # the limit is part of the captured launch
    finally:
        scan.set_spin_limit(0)
        scan.force_config(-1)
    statuses = []
    try:
        for _ in range(8):
            s = L.scan_graph_launch(g._h, stream())
            torch.cuda.synchronize()
            statuses.append(s)
            if s == TIMEOUT:
                break
        assert statuses[-1] == TIMEOUT, statuses
        assert all(s == 0 for s in statuses[:-1]), statuses
        # the explicit check of a replay that has finished
        check_status(L.scan_graph_launch(g._h, stream()))
        torch.cuda.synchronize()
        assert L.scan_graph_check_device_error(g._h) in (0, TIMEOUT)
        assert L.scan_graph_check_device_error(g._h) == 0       # cleared by the read
    finally:
        g.close()
    # a graph created with the default limit is exact
    g = scan.SegmentedScanGraph(x, y, offs)
    g.launch()
    torch.cuda.synchronize()
    assert not first_mismatch(y.cpu().numpy().view(np.uint32), oracle.segmented_int(a, off))
    g.close()
