"""The streaming-ceiling kernel (the scan's memory access pattern without the
scan, used by the bench as the roofline of the access pattern): for every
counter-mode configuration it writes out = in + 1 modulo 2^32 over ragged
sizes, in place and out of place, and leaves the stream's workspace usable
for the scans that follow."""
import numpy as np
import pytest

import oracle
from gpu_util import check_status, lib, stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _counter_configs():
    from paper_2312_14874_amd import config_info, num_configs
    return [c for c in range(num_configs()) if config_info(c)["mode"] in (0, 1)]


@pytest.mark.parametrize("n", [1, 4097, 98304 * 3 + 5, (1 << 22) + 11])
def test_ceiling_kernel_adds_one_everywhere(n):
    L = lib()
    g = np.random.default_rng(7600 + n % 97)
    a = g.integers(0, 1 << 32, size=n, dtype=np.uint32)
    a[: min(n, 3)] = 0xFFFFFFFF                      # wraps to 0
    x = torch.from_numpy(a.view(np.int32)).cuda()
    want = a + np.uint32(1)
    for cfg in _counter_configs():
        y = torch.empty_like(x)
        print("ceiling config %d n=%d" % (cfg, n), flush=True)
        check_status(L.scan_stream_ceiling(x.data_ptr(), y.data_ptr(), n, cfg, stream()), "scan_stream_ceiling")
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint32), want), "config %d" % cfg
    z = x.clone()
    check_status(L.scan_stream_ceiling(z.data_ptr(), z.data_ptr(), n, 22, stream()), "in place")
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy().view(np.uint32), want)
    # the workspace it shares with the scans is left clean
    y = torch.empty_like(x)
    check_status(L.scan_flat(x.data_ptr(), y.data_ptr(), n, 1, 0, stream()), "scan_flat")
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().view(np.uint32), oracle.scan_int(a))
