"""Two-way partition (the compaction kernel with the rejected elements written
to the end of the output in reverse order) against the oracle, bit-exact: both
predicates, the three dtypes, selectivities from none to all, ragged sizes,
misaligned input, and the 2^28 workload size."""
import numpy as np
import pytest

import oracle
from gpu_util import DT, check_status, first_mismatch, from_dev, lib, stream, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRED = {"nonzero": 0, "greater": 1}
TILE = 1024 * 64   # the partition kernel's tile
OLD_TILE = 256 * 64


def run(a, predicate, threshold=0, misalign=0):
    L = lib()
    x = to_dev(a, pad=misalign + 4)
    xin = x[misalign + 4:]
    out = torch.full((a.size + 8,), -1, dtype=torch.int32, device="cuda").view(x.dtype)   # guard bits all ones
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    thr = int(np.array([threshold], dtype=a.dtype).view(np.uint32)[0])
    check_status(L.scan_partition(xin.data_ptr(), out[4:].data_ptr(), a.size, DT[a.dtype], PRED[predicate], thr,
                                  cnt.data_ptr(), stream()), "scan_partition n=%d" % a.size)
    torch.cuda.synchronize()
    res = from_dev(out, a.dtype)
    # nothing written outside out[0 .. n)
    guard = res.view(np.uint32)
    assert np.all(guard[:4] == 0xFFFFFFFF) and np.all(guard[4 + a.size:] == 0xFFFFFFFF)
    return res[4:4 + a.size], int(cnt.item())


def data(n, seed, dtype, zero_frac=0.5):
    g = np.random.default_rng(seed)
    if dtype == np.float32:
        a = g.standard_normal(n).astype(np.float32)
    else:
        a = g.integers(np.iinfo(dtype).min, np.iinfo(dtype).max, size=n, dtype=np.int64, endpoint=True).astype(dtype)
    a[g.random(n) < zero_frac] = 0
    return a


def check(a, predicate, threshold=0, **kw):
    want, k_want = oracle.partition(a, predicate, threshold)
    got, k = run(a, predicate, threshold, **kw)
    assert k == k_want, (k, k_want)
    err = first_mismatch(got.view(np.uint32), np.asarray(want).view(np.uint32))
    assert not err, "n=%d: %s" % (a.size, err)


@pytest.mark.parametrize("dtype", [np.int32, np.uint32, np.float32])
@pytest.mark.parametrize("n", [1, 2, 100, 255, 257, OLD_TILE - 1, OLD_TILE + 1, TILE - 1, TILE, TILE + 1, 5 * TILE + 777,
                               (1 << 20) + 9])
def test_nonzero(dtype, n):
    check(data(n, 7300 + n % 83, dtype), "nonzero")


@pytest.mark.parametrize("dtype,thr", [(np.int32, 0), (np.int32, -1 << 30), (np.uint32, 1 << 31),
                                       (np.float32, 0.5), (np.float32, -3.0)])
def test_greater(dtype, thr):
    check(data(3 * TILE + 99, 7400, dtype, zero_frac=0.1), "greater", thr)


# several tiles with a ragged last one: past n the loads read zeros, which a
# signed or float compare with a negative threshold would keep
@pytest.mark.parametrize("dtype,thr", [(np.int32, -1 << 30), (np.int32, -1), (np.float32, -3.0), (np.uint32, 0)])
@pytest.mark.parametrize("n", [5 * TILE + 777, 3 * TILE + 4096 * 7 + 1283])
def test_greater_ragged_tiles(dtype, thr, n):
    check(data(n, 4150 + n % 97, dtype, zero_frac=0.1), "greater", thr)


# thresholds at the ends of each type's range, with those values (and, for
# float32, infinities, NaN and both zeros) in the data; several tiles and a
# ragged last one, where the elements past n read as a value never kept
@pytest.mark.parametrize("dtype,thr", [(np.int32, int(np.iinfo(np.int32).min)), (np.int32, int(np.iinfo(np.int32).max)),
                                       (np.uint32, 0), (np.uint32, int(np.iinfo(np.uint32).max)),
                                       (np.float32, -np.inf), (np.float32, np.inf), (np.float32, np.nan)])
def test_greater_extreme_thresholds(dtype, thr):
    a = data(4 * TILE + 3 * 4096 + 517, 4160, dtype, zero_frac=0.1)
    if dtype == np.float32:
        specials = np.array([np.inf, -np.inf, np.nan, 0.0, -0.0], dtype=np.float32)
    else:
        info = np.iinfo(dtype)
        specials = np.array([info.min, info.max, 0, 1, info.max - 1], dtype=dtype)
    a[::97] = np.resize(specials, a[::97].size)
    check(a, "greater", thr)


@pytest.mark.parametrize("zero_frac", [0.0, 1.0, 0.999, 0.001])
def test_selectivity_extremes(zero_frac):
    check(data(7 * TILE + 5, 7500, np.int32, zero_frac=zero_frac), "nonzero")


def test_nan_rejected():
    a = data(50000, 7600, np.float32)
    a[::7] = np.nan
    check(a, "greater", -1e30)


def test_misaligned():
    a = data(9 * TILE + 321, 7700, np.int32)
    for mis in (1, 2, 3):
        check(a, "nonzero", misalign=mis)


def test_zero_length_writes_count():
    L = lib()
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    check_status(L.scan_partition(None, None, 0, 0, 0, 0, cnt.data_ptr(), stream()), "scan_partition n=0")
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


def test_torch_binding():
    import paper_2312_14874_amd as m
    a = data(4 * TILE + 3, 7800, np.int32)
    out, k = m.partition(torch.from_numpy(a).cuda(), "greater", 0)
    want, k_want = oracle.partition(a, "greater", 0)
    assert k == k_want and not first_mismatch(out.cpu().numpy(), np.asarray(want))


def test_full_size():
    a = data(1 << 28, 7900, np.int32, zero_frac=0.5)
    check(a, "greater", 0)


def test_beyond_2p30_elements():
    # byte offsets past 2^32: the output ranges are addressed from per-wave bases
    n = (1 << 30) + 7
    a = data(n, 8000, np.uint32, zero_frac=0.3)
    check(a, "nonzero")
