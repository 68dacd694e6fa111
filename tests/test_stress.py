"""Repeated launches (the test pyramid's stress level): the smallest tiles,
every configuration whose tile order relies on in-order dispatch (mode 2) and
random configurations, hundreds of launches each on one stream, so that the
self-cleaning workspace flips parity hundreds of times and ordered launches
alternate with counter-mode ones.  Every result is checked bit-exact against
the oracle and the run stops at the first mismatch."""
import numpy as np
import pytest

import oracle
from gpu_util import check_status, lib, stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REPS = 200


def _configs():
    from paper_2312_14874_amd import config_info, num_configs
    infos = [config_info(c) for c in range(num_configs())]
    smallest = min(i["tile"] for i in infos)
    ordered = [i["config"] for i in infos if i["mode"] == 2]
    small = [i["config"] for i in infos if i["tile"] == smallest]
    return sorted(set(ordered + small)), infos


def _run(L, x, y, n, flags, cfg, seg_off=None, S=0):
    check_status(L.scan_force_config(cfg))
    try:
        if seg_off is None:
            check_status(L.scan_flat(x.data_ptr(), y.data_ptr(), n, 0, flags, stream()), "scan_flat")
        else:
            check_status(L.scan_segmented_batch(x.data_ptr(), y.data_ptr(), seg_off.data_ptr(), S, n, 0, flags,
                                                stream()), "scan_segmented_batch")
    finally:
        L.scan_force_config(-1)


def test_repeated_launches_smallest_tiles_and_ordered_configs():
    L = lib()
    cfgs, infos = _configs()
    g = np.random.default_rng(7500)
    big = g.integers(-(1 << 31), (1 << 31) - 1, size=1 << 21, dtype=np.int64).astype(np.int32)
    xd = torch.from_numpy(big).cuda()
    y = torch.empty_like(xd)
    for cfg in cfgs:
        tile = infos[cfg]["tile"]
        for rep in range(REPS):
            n = int(g.integers(2 * tile, min(big.size, 64 * tile)))
            lo = int(g.integers(0, big.size - n + 1)) & ~3        # 16-byte aligned start
            n = min(n, big.size - lo)
            flags = int(g.integers(0, 2))
            _run(L, xd[lo:], y, n, flags, cfg)
            got = y[:n].cpu().numpy()
            want = oracle.scan_int(big[lo:lo + n], exclusive=bool(flags))
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, "config %d rep %d n=%d flags=%d: first mismatch at %d" % (cfg, rep, n, flags, bad[0])
    assert L.scan_check_device_error(stream()) == 0


def test_repeated_launches_random_configs_flat_and_segmented():
    L = lib()
    from paper_2312_14874_amd import num_configs
    import workloads
    g = np.random.default_rng(7501)
    big = g.integers(0, 1 << 32, size=1 << 21, dtype=np.uint32).view(np.int32)
    xd = torch.from_numpy(big).cuda()
    y = torch.empty_like(xd)
    for rep in range(2 * REPS):
        cfg = int(g.integers(0, num_configs()))
        n = int(g.integers(1, big.size))
        flags = int(g.integers(0, 4))                              # exclusive and / or reverse
        if rep % 2:
            S = int(g.integers(1, 200))
            off = workloads.random_offsets(g, n, S)
            offs = torch.from_numpy(off).cuda()
            _run(L, xd, y, n, flags, cfg, offs, S)
            want = oracle.segmented_int(big[:n], off, exclusive=bool(flags & 1), reverse=bool(flags & 2))
        else:
            _run(L, xd, y, n, flags, cfg)
            want = oracle.scan_int(big[:n], exclusive=bool(flags & 1), reverse=bool(flags & 2))
        got = y[:n].cpu().numpy()
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, "rep %d config %d n=%d flags=%d seg=%d: first mismatch at %d" % (
            rep, cfg, n, flags, rep % 2, bad[0])
    assert L.scan_check_device_error(stream()) == 0
