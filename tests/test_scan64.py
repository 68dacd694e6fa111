"""64-bit scans (scan_flat with SCAN_I64 / SCAN_U64 / SCAN_F64) against the
oracle: integers bit-exact, float64 within the summation bound; ragged sizes
across tile boundaries, inclusive and exclusive, forward and reverse, in
place, carries out of the low 32 bits, wrap-around modulo 2^64, a workspace
shared with 32-bit scans on one stream, autograd, and 2^28 elements."""
import numpy as np
import pytest

import oracle
from gpu_util import check_status, first_mismatch, flat, lib, stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

I64, U64 = 3, 4
TILE = 512 * 64   # elements per tile of the 64-bit kernel


def to_dev64(a: np.ndarray, pad: int = 2) -> torch.Tensor:
    """int64 device copy with `pad` spare elements in front (2 keeps 16-byte alignment)."""
    t = torch.empty(a.size + pad, dtype=torch.int64, device="cuda")
    t[pad:].copy_(torch.from_numpy(np.ascontiguousarray(a).view(np.int64)))
    return t[pad:]


def run64(a: np.ndarray, exclusive=False, inplace=False, reverse=False) -> np.ndarray:
    x = to_dev64(a)
    out = x if inplace else to_dev64(np.zeros(a.size, dtype=np.int64))
    dt = U64 if a.dtype == np.uint64 else I64
    flags = (1 if exclusive else 0) | (2 if reverse else 0)
    check_status(lib().scan_flat(x.data_ptr(), out.data_ptr(), a.size, dt, flags, stream()),
                 "scan_flat n=%d" % a.size)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(a.dtype)


def data(n, seed, dtype=np.uint64, kind="uniform"):
    g = np.random.default_rng(seed)
    if kind == "uniform":        # the whole 64-bit range: wraps at almost every step
        a = g.integers(0, 1 << 64, size=n, dtype=np.uint64)
    elif kind == "carry":        # low halves near 2^32: a carry into the high half at most steps
        a = (np.uint64(0xFFFFFFFF) - g.integers(0, 16, size=n, dtype=np.uint64))
    else:                        # small signed values: sums stay near zero
        a = g.integers(-1000, 1000, size=n, dtype=np.int64).view(np.uint64)
    return a.view(dtype)


def check(a, exclusive=False, reverse=False, **kw):
    want = oracle.scan_int64(a, exclusive=exclusive, reverse=reverse)
    got = run64(a, exclusive, reverse=reverse, **kw)
    assert got.dtype == a.dtype
    err = first_mismatch(got.view(np.uint64), want.view(np.uint64))
    assert not err, "n=%d ex=%d rev=%d: %s" % (a.size, exclusive, reverse, err)


@pytest.mark.parametrize("n", [1, 2, 3, 127, 128, 129, TILE - 1, TILE, TILE + 1, 5 * TILE + 777, (1 << 20) + 3])
@pytest.mark.parametrize("exclusive", [False, True])
@pytest.mark.parametrize("reverse", [False, True])
def test_ragged(n, exclusive, reverse):
    check(data(n, 6000 + n % 97), exclusive, reverse)


@pytest.mark.parametrize("kind", ["uniform", "carry", "small"])
@pytest.mark.parametrize("dtype", [np.int64, np.uint64])
def test_value_patterns(kind, dtype):
    check(data(37 * TILE + 4099, 6100, dtype, kind), exclusive=False)
    check(data(37 * TILE + 4099, 6101, dtype, kind), exclusive=True)


def test_in_place():
    check(data(11 * TILE + 5, 6200), inplace=True)
    check(data(11 * TILE + 5, 6201), exclusive=True, inplace=True)
    check(data(11 * TILE + 5, 6202), reverse=True, inplace=True)


def test_shares_workspace_with_32bit_scans():
    # the stream's status words alternate between the two protocols (one word
    # per 32-bit tile, two per 64-bit tile) and between large and small calls
    g = np.random.default_rng(6300)
    for step, (bits, n) in enumerate([(32, 1 << 26), (64, 1 << 22), (32, 1 << 26), (64, 1 << 26),
                                      (32, 1 << 20), (64, 3 * TILE + 1), (64, 1 << 25), (32, 1 << 24)]):
        if bits == 32:
            a = g.integers(0, 1 << 32, size=n, dtype=np.uint32)
            err = first_mismatch(flat(a), np.asarray(oracle.scan_int(a)))
        else:
            a = data(n, 6400 + step)
            err = first_mismatch(run64(a), oracle.scan_int64(a))
        assert not err, "step %d (%d-bit, n=%d): %s" % (step, bits, n, err)


def test_torch_binding():
    import paper_2312_14874_amd as m
    a = data(3 * TILE + 17, 6500, np.int64, "small")
    x = torch.from_numpy(a).cuda()
    assert x.data_ptr() % 16 == 0
    got = m.cumsum(x).cpu().numpy()
    assert not first_mismatch(got, oracle.scan_int64(a))
    got = m.cumsum(x, exclusive=True).cpu().numpy()
    assert not first_mismatch(got, oracle.scan_int64(a, exclusive=True))
    got = m.cumsum(x, reverse=True).cpu().numpy()
    assert not first_mismatch(got, oracle.scan_int64(a, reverse=True))
    with pytest.raises(m.ScanError):
        m.cumsum(x, op="max")


def test_full_size():
    check(data(1 << 28, 6600), exclusive=False)
    check(data(1 << 28, 6601), exclusive=True, reverse=True)


# ---------------------------------------------------------------- float64

F64 = 5


def run_f64(a: np.ndarray, exclusive=False, inplace=False, reverse=False) -> np.ndarray:
    x = torch.empty(a.size + 2, dtype=torch.float64, device="cuda")[2:]
    x.copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)))
    out = x if inplace else torch.zeros(a.size + 2, dtype=torch.float64, device="cuda")[2:]
    flags = (1 if exclusive else 0) | (2 if reverse else 0)
    check_status(lib().scan_flat(x.data_ptr(), out.data_ptr(), a.size, F64, flags, stream()),
                 "scan_flat f64 n=%d" % a.size)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_f64(a, exclusive=False, reverse=False, **kw):
    """Within the recursive-summation bound of the kernel's addition tree: at
    most 8 levels per tile of the look-back chain plus 128 inside a tile."""
    ref, ab = oracle.scan_f64(a, exclusive=exclusive, reverse=reverse)
    got = run_f64(a, exclusive, reverse=reverse, **kw)
    depth = 8 * (-(-a.size // TILE)) + 128
    tol = oracle.f64_tolerance(ab, depth)
    err = np.abs(got - ref)
    bad = np.nonzero(~(err <= tol))[0]
    assert bad.size == 0, "n=%d ex=%d: %d out of bound, first %d: got %r want %r tol %r" % (
        a.size, exclusive, bad.size, bad[0], got[bad[0]], ref[bad[0]], tol[bad[0]])


def normal_f64(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("n", [1, 2, 3, 129, TILE - 1, TILE, TILE + 1, 5 * TILE + 777, (1 << 20) + 3])
@pytest.mark.parametrize("exclusive", [False, True])
@pytest.mark.parametrize("reverse", [False, True])
def test_f64_ragged(n, exclusive, reverse):
    check_f64(normal_f64(n, 6700 + n % 89), exclusive, reverse)


def test_f64_values():
    g = np.random.default_rng(6800)
    n = 23 * TILE + 1001
    # integer-valued (every partial sum exact in any order): equal to the oracle
    a = g.integers(-1000, 1001, size=n).astype(np.float64)
    assert not first_mismatch(run_f64(a), oracle.scan_f64(a)[0])
    # wide exponent range, and cancelling pairs
    check_f64(g.standard_normal(n) * np.ldexp(1.0, g.integers(-40, 40, size=n)))
    b = g.standard_normal(n)
    b[1::2] = -b[0::2][: b[1::2].size]
    check_f64(b, exclusive=True)


def test_f64_in_place():
    check_f64(normal_f64(9 * TILE + 3, 6900), inplace=True)
    check_f64(normal_f64(9 * TILE + 3, 6901), reverse=True, inplace=True)


def test_f64_autograd_gradcheck():
    # the backward of the float64 cumsum is the reverse scan: torch's
    # numerical Jacobian check, on a size that spans several tiles
    import paper_2312_14874_amd as m
    g = torch.Generator().manual_seed(7050)
    x = torch.randn(2 * TILE + 17, generator=g, dtype=torch.float64).cuda().requires_grad_()
    y = m.cumsum_autograd(x)
    gy = torch.randn(x.numel(), generator=g, dtype=torch.float64).cuda()
    (gx,) = torch.autograd.grad(y, x, gy)
    ref, ab = oracle.scan_f64(gy.cpu().numpy(), reverse=True)
    tol = oracle.f64_tolerance(ab, 8 * 3 + 128)
    assert np.all(np.abs(gx.cpu().numpy() - ref) <= tol)
    small = torch.randn(300, generator=g, dtype=torch.float64).cuda().requires_grad_()
    assert torch.autograd.gradcheck(m.cumsum_autograd, (small,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_f64_torch_binding():
    import paper_2312_14874_amd as m
    a = normal_f64(4 * TILE + 5, 7000)
    x = torch.from_numpy(a).cuda()
    got = m.cumsum(x).cpu().numpy()
    ref, ab = oracle.scan_f64(a)
    assert np.all(np.abs(got - ref) <= oracle.f64_tolerance(ab, 8 * 5 + 128))


def test_f64_full_size():
    check_f64(normal_f64(1 << 28, 7100))
    check_f64(normal_f64(1 << 28, 7101), exclusive=True, reverse=True)


def test_capture_mixed_widths_after_reserve():
    """A caller's graph holding a uint64 scan, a float64 reverse scan and a
    32-bit scan on one stream's reserved workspace, replayed with eager calls
    of the other widths on the same stream in between."""
    import paper_2312_14874_amd as m
    n = 3 * TILE * 5 + 77
    g = np.random.default_rng(7200)
    a64 = g.integers(0, 1 << 64, size=n, dtype=np.uint64)
    f = g.standard_normal(n)
    a32 = g.integers(-1 << 31, 1 << 31, size=4 * n, dtype=np.int64).astype(np.int32)
    x64, xf, x32 = (torch.from_numpy(v).cuda() for v in (a64.view(np.int64), f, a32))
    y64, yf, y32 = torch.empty_like(x64), torch.empty_like(xf), torch.empty_like(x32)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        m.reserve(4 * n)
        m.cumsum(x64, out=y64)
        m.cumsum(xf, reverse=True, out=yf)
        m.cumsum(x32, out=y32)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        m.cumsum(x64, out=y64)
        m.cumsum(xf, reverse=True, out=yf)
        m.cumsum(x32, out=y32)
    w64 = oracle.scan_int64(a64)
    wf, ab = oracle.scan_f64(f, reverse=True)
    w32 = oracle.scan_int(a32)
    tol = oracle.f64_tolerance(ab, 8 * (-(-n // TILE)) + 128)
    e64 = torch.empty_like(x64)
    for rep in range(4):
        for t in (y64, yf, y32):
            t.zero_()
        with torch.cuda.stream(s):
            graph.replay()
            m.cumsum(x32, exclusive=True, out=torch.empty_like(x32))   # eager, same workspace
            m.cumsum(x64, exclusive=True, out=e64)
        torch.cuda.synchronize()
        assert not first_mismatch(y64.cpu().numpy().view(np.uint64), w64), rep
        assert np.all(np.abs(yf.cpu().numpy() - wf) <= tol), rep
        assert not first_mismatch(y32.cpu().numpy(), w32), rep
        assert not first_mismatch(e64.cpu().numpy().view(np.uint64), oracle.scan_int64(a64, exclusive=True)), rep


def test_beyond_2p32_bytes():
    # 2^29 + 3 uint64 elements: 4 GiB per buffer, byte offsets past 2^32
    check(data((1 << 29) + 3, 8100), exclusive=False)
