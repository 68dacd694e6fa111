"""hipGraph capture and replay of the batched segmented scan and of the
per-segment-launch comparator.  Every replay is checked against the oracle,
with eager work and synchronisations between replays, and new input data
under a fixed graph must give new correct results."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import first_mismatch, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _case(seed, n, S):
    g = np.random.default_rng(seed)
    a = workloads.full_u32(n, seed=seed)
    off = workloads.random_offsets(g, n, S)
    return a, off


@pytest.mark.parametrize("n,S", [(1000, 5), (3_000_001, 700), (40_000_000, 4096)])
def test_segmented_graph_replays(n, S):
    _graph_replays(n, S)


# the graph captures the configuration chosen at creation: the large-tile
# segmented kernels, plain (21) and with early publication (35)
@pytest.mark.parametrize("cfg", [21, 35])
def test_segmented_graph_replays_config(cfg):
    _graph_replays(3_000_001, 700, cfg)


def _graph_replays(n, S, cfg=None):
    import paper_2312_14874_amd as scan
    a, off = _case(n, n, S)
    x = to_dev(a)
    out = torch.empty_like(x)
    offs = torch.from_numpy(off).cuda()
    if cfg is not None:
        scan.force_config(cfg)
    try:
        g = scan.SegmentedScanGraph(x, out, offs, exclusive=True)
    finally:
        if cfg is not None:
            scan.force_config(-1)
    want = oracle.segmented_int(a, off, exclusive=True)
    for rep in range(5):
        out.zero_()
        g.launch()
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert not first_mismatch(got, want), "replay %d" % rep
        # eager work between replays on the same stream
        scan.cumsum(x[:1000].clone())
        torch.cuda.synchronize()
    # new contents, same buffers
    b = workloads.full_u32(n, seed=n + 1)
    x.copy_(torch.from_numpy(b.view(np.int32)))
    g.launch()
    torch.cuda.synchronize()
    assert not first_mismatch(out.cpu().numpy().view(np.uint32), oracle.segmented_int(b, off, exclusive=True))
    g.close()


def test_segmented_graph_f32_reverse():
    import paper_2312_14874_amd as scan
    n = 2_000_003
    a = workloads.normal_f32(n, seed=9)
    off = workloads.random_offsets(np.random.default_rng(9), n, 64)
    x = torch.from_numpy(a).cuda()
    out = torch.empty_like(x)
    g = scan.SegmentedScanGraph(x, out, torch.from_numpy(off).cuda(), reverse=True)
    ref, ab = oracle.segmented_f32(a, off, reverse=True)
    tol = np.ldexp(ab, -20)
    first = None
    for _ in range(3):
        g.launch()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.abs(got.astype(np.float64) - ref) <= tol)
        if first is None:
            first = got.copy()
        assert np.array_equal(first.view(np.uint32), got.view(np.uint32))   # deterministic
    g.close()


def test_looped_graph_matches_batched():
    import paper_2312_14874_amd as scan
    n, S = 2_000_000, 300
    a, off = _case(77, n, S)
    x = to_dev(a)
    out_l = torch.empty_like(x)
    out_b = torch.empty_like(x)
    gl = scan.LoopedScanGraph(x, out_l, off, exclusive=True)
    for _ in range(3):
        gl.launch()
    scan.segmented_scan(x, torch.from_numpy(off).cuda(), exclusive=True, out=out_b)
    torch.cuda.synchronize()
    want = oracle.segmented_int(a, off, exclusive=True)
    assert not first_mismatch(out_l.cpu().numpy().view(np.uint32), want)
    assert not first_mismatch(out_b.cpu().numpy().view(np.uint32), want)
    gl.close()


def test_looped_eager_matches_oracle():
    import paper_2312_14874_amd as scan
    n, S = 1_500_000, 257
    a, off = _case(78, n, S)
    x = to_dev(a)
    out = scan.segmented_scan_looped(x, off, exclusive=False)
    torch.cuda.synchronize()
    assert not first_mismatch(out.cpu().numpy().view(np.uint32), oracle.segmented_int(a, off))


def test_capture_of_flat_scan_after_reserve():
    """Library calls captured by the caller into its own graph (workspace reserved first)."""
    import paper_2312_14874_amd as scan
    n = 5_000_000
    a = workloads.full_u32(n, seed=5)
    x = to_dev(a)
    out = torch.empty_like(x)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        scan.reserve(n)
        scan.cumsum(x, out=out)   # warm: workspace exists for this stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        scan.cumsum(x, out=out)
    want = oracle.scan_int(a)
    for _ in range(4):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert not first_mismatch(out.cpu().numpy().view(np.uint32), want)


def test_captured_graph_survives_workspace_growth():
    """A graph captured from library calls keeps its workspace when a later,
    larger eager call on the same stream grows the stream's workspace."""
    import paper_2312_14874_amd as scan
    n = 3_000_000
    a = workloads.full_u32(n, seed=15)
    x = to_dev(a)
    out = torch.empty_like(x)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        scan.reserve(n)
        scan.cumsum(x, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        scan.cumsum(x, out=out)
    want = oracle.scan_int(a)
    # an eager call needing many more tiles than reserved: 4096-element tiles
    big = workloads.full_u32(16 * n, seed=16)
    xb = to_dev(big)
    yb = torch.empty_like(xb)
    scan.force_config(11)
    try:
        with torch.cuda.stream(s):
            scan.cumsum(xb, out=yb)
    finally:
        scan.force_config(-1)
    torch.cuda.synchronize()
    assert not first_mismatch(yb.cpu().numpy().view(np.uint32), oracle.scan_int(big))
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert not first_mismatch(out.cpu().numpy().view(np.uint32), want)
        with torch.cuda.stream(s):
            scan.cumsum(xb, out=yb)        # eager work on the grown workspace in between
        torch.cuda.synchronize()
    assert not first_mismatch(yb.cpu().numpy().view(np.uint32), oracle.scan_int(big))


def test_looped_graph_with_misaligned_segments():
    """Segments whose start is not 16-byte aligned take the dword kernel's
    smaller tiles: the graph's workspace is sized for those."""
    import paper_2312_14874_amd as scan
    for off in (np.array([0, 3, 20003], dtype=np.int64), np.array([0, 1, 5, 70_006, 70_007], dtype=np.int64)):
        n = int(off[-1])
        a = workloads.full_u32(n, seed=n)
        x = to_dev(a)
        out = torch.empty_like(x)
        gl = scan.LoopedScanGraph(x, out, off, exclusive=True)
        gl.launch()
        torch.cuda.synchronize()
        assert not first_mismatch(out.cpu().numpy().view(np.uint32), oracle.segmented_int(a, off, exclusive=True))
        gl.close()
