"""Failure handling of the look-back's bounded wait, forced from the host: with
a spin limit of one poll, a tile that has to wait gives up, marks the
workspace's error word and the kernel finishes normally (results of that call
invalid); scan_check_device_error reports SCAN_ERROR_TIMEOUT once and clears
the word; with the default limit restored the next scans are exact again.
Only scans take part, whose addresses never depend on the values a timed-out
look-back leaves wrong."""
import numpy as np
import pytest

import oracle
from gpu_util import check_status, first_mismatch, flat, lib, stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TIMEOUT = 7


def test_spin_limit_timeout_is_reported_and_cleared():
    L = lib()
    g = np.random.default_rng(7200)
    a32 = g.integers(0, 1 << 32, size=1 << 26, dtype=np.uint32)
    a64 = g.integers(0, 1 << 64, size=1 << 25, dtype=np.uint64)
    x64 = torch.from_numpy(a64.view(np.int64)).cuda()
    y64 = torch.empty_like(x64)
    seen = []
    check_status(L.scan_set_spin_limit(1))
    try:
        for _ in range(4):
            flat(a32)                                   # launches must still succeed
            seen.append(L.scan_check_device_error(stream()))
            check_status(L.scan_flat(x64.data_ptr(), y64.data_ptr(), a64.size, 4, 0, stream()), "scan_flat u64")
            seen.append(L.scan_check_device_error(stream()))
    finally:
        check_status(L.scan_set_spin_limit(0))
    assert all(s in (0, TIMEOUT) for s in seen), seen
    print("timeouts reported: %d of %d calls" % (seen.count(TIMEOUT), len(seen)))
    # the error word was cleared by each check, and the workspace still works
    assert L.scan_check_device_error(stream()) == 0
    assert not first_mismatch(flat(a32), np.asarray(oracle.scan_int(a32)))
    check_status(L.scan_flat(x64.data_ptr(), y64.data_ptr(), a64.size, 4, 0, stream()), "scan_flat u64")
    torch.cuda.synchronize()
    assert not first_mismatch(y64.cpu().numpy().view(np.uint64), oracle.scan_int64(a64))
    assert L.scan_check_device_error(stream()) == 0
