"""The autotuner on the GPU (scan_autotune, Section 4.2.4's partition-size
sweep on the GPU's tile configurations): it times every configuration at the
call's size, stores the winner for the call's (dtype, segmented, log2 n)
bucket, the library then selects it for that bucket, and scans under it equal
the oracle.  The shipped table is reloaded afterwards."""
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_f32_close

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _shipped():
    import paper_2312_14874_amd as scan
    return os.path.join(os.path.dirname(scan.LIB_PATH), "tune", "gfx950.json")


@pytest.mark.parametrize("seg", [False, True])
@pytest.mark.parametrize("dtype", [torch.int32, torch.float32])
def test_autotune_stores_selects_and_scans_exactly(seg, dtype):
    import paper_2312_14874_amd as scan
    n = 3 * 98304 + 77
    g = np.random.default_rng(7400 + 2 * int(seg) + (dtype == torch.float32))
    a = workloads.normal_f32(n, seed=7401) if dtype == torch.float32 else \
        g.integers(-1000, 1000, size=n, dtype=np.int32)
    x = torch.from_numpy(a).cuda()
    y = torch.empty_like(x)
    off = workloads.random_offsets(g, n, 37) if seg else None
    offs = torch.from_numpy(off).cuda() if seg else None
    before = scan.selected_config(dtype, n, segmented=seg)
    try:
        best = scan.autotune(x, y, offsets=offs, reps=2)
        assert 0 <= best < scan.num_configs()
        assert scan.selected_config(dtype, n, segmented=seg) == best
        # another size in the same bucket selects it too
        assert scan.selected_config(dtype, n + 1000, segmented=seg) == best
        info = scan.config_info(best)
        print("autotune seg=%s %s n=%d: config %d %s" % (seg, dtype, n, best, info), flush=True)
        got = (scan.segmented_scan(x, offs) if seg else scan.cumsum(x)).cpu().numpy()
        if dtype == torch.int32:
            want = oracle.segmented_int(a, off) if seg else oracle.scan_int(a)
            assert np.array_equal(got, want)
        else:
            ref, ab = oracle.segmented_f32(a, off) if seg else oracle.scan_f32(a)
            assert_f32_close(got, ref, ab)
    finally:
        scan.tune_load(_shipped())
    assert scan.selected_config(dtype, n, segmented=seg) == before
