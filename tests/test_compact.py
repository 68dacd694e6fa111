"""Stream compaction fused with the exclusive scan against the oracle, bit-exact:
both predicates, the three dtypes, selectivities from none to all, ragged
sizes, in place, misaligned input, and the 2^28 workload size."""
import numpy as np
import pytest

import oracle
from gpu_util import DT, check_status, first_mismatch, from_dev, lib, stream, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRED = {"nonzero": 0, "greater": 1}


def run(a, predicate, threshold=0, misalign=0, inplace=False):
    L = lib()
    x = to_dev(a, pad=misalign + 4)
    xin = x[misalign + 4:]
    out = xin if inplace else torch.full((a.size + 4,), -1, dtype=x.dtype, device="cuda")[4:]
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    thr = int(np.array([threshold], dtype=a.dtype).view(np.uint32)[0])
    check_status(L.scan_compact(xin.data_ptr(), out.data_ptr(), a.size, DT[a.dtype], PRED[predicate], thr,
                                cnt.data_ptr(), stream()), "scan_compact")
    torch.cuda.synchronize()
    k = int(cnt.item())
    return from_dev(out, a.dtype)[:k], k


def data(n, seed, dtype, zero_frac=0.5):
    g = np.random.default_rng(seed)
    if dtype == np.float32:
        a = g.standard_normal(n).astype(np.float32)
    else:
        a = g.integers(np.iinfo(dtype).min, np.iinfo(dtype).max, size=n, dtype=np.int64, endpoint=True).astype(dtype)
    a[g.random(n) < zero_frac] = 0
    return a


def check(a, predicate, threshold=0, **kw):
    want = oracle.compact(a, predicate, threshold)
    got, k = run(a, predicate, threshold, **kw)
    assert k == want.size, (k, want.size)
    assert not first_mismatch(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("dtype", [np.int32, np.uint32, np.float32])
# tile edges of the compaction kernel (1024 threads x 64 elements) and of an
# earlier 16384-element shape, ragged chunk and lane ends
@pytest.mark.parametrize("n", [1, 100, 255, 257, 16383, 16384, 16385, 5 * 16384 + 777, 65535, 65536, 65537,
                               3 * 65536 + 4095, 1 << 20, (1 << 20) + 13])
def test_nonzero(dtype, n):
    check(data(n, 4000 + n % 89, dtype), "nonzero")


@pytest.mark.parametrize("dtype,thr", [(np.int32, 0), (np.int32, -1 << 30), (np.uint32, 1 << 31),
                                       (np.float32, 0.5), (np.float32, -3.0)])
def test_greater(dtype, thr):
    check(data(3 * 16384 + 99, 4100, dtype, zero_frac=0.1), "greater", thr)


# several tiles with a ragged last one: past n the loads read zeros, which a
# signed or float compare with a negative threshold would keep
@pytest.mark.parametrize("dtype,thr", [(np.int32, -1 << 30), (np.int32, -1), (np.float32, -3.0), (np.uint32, 0)])
@pytest.mark.parametrize("n", [5 * 65536 + 777, 3 * 65536 + 4096 * 7 + 1283])
def test_greater_ragged_tiles(dtype, thr, n):
    check(data(n, 4150 + n % 97, dtype, zero_frac=0.1), "greater", thr)


# thresholds at the ends of each type's range, with those values (and, for
# float32, infinities, NaN and both zeros) in the data; several tiles and a
# ragged last one, where the elements past n read as a value never kept
@pytest.mark.parametrize("dtype,thr", [(np.int32, int(np.iinfo(np.int32).min)), (np.int32, int(np.iinfo(np.int32).max)),
                                       (np.uint32, 0), (np.uint32, int(np.iinfo(np.uint32).max)),
                                       (np.float32, -np.inf), (np.float32, np.inf), (np.float32, np.nan)])
def test_greater_extreme_thresholds(dtype, thr):
    a = data(4 * 65536 + 3 * 4096 + 517, 4160, dtype, zero_frac=0.1)
    if dtype == np.float32:
        specials = np.array([np.inf, -np.inf, np.nan, 0.0, -0.0], dtype=np.float32)
    else:
        info = np.iinfo(dtype)
        specials = np.array([info.min, info.max, 0, 1, info.max - 1], dtype=dtype)
    a[::97] = np.resize(specials, a[::97].size)
    check(a, "greater", thr)


@pytest.mark.parametrize("zero_frac", [0.0, 1.0, 0.999, 0.001])
def test_selectivity_extremes(zero_frac):
    check(data(7 * 16384 + 5, 4200, np.int32, zero_frac=zero_frac), "nonzero")


def test_nan_never_kept():
    a = data(50000, 4300, np.float32)
    a[::7] = np.nan
    check(a, "greater", -1e30)


def test_zero_length_writes_count():
    L = lib()
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    check_status(L.scan_compact(None, None, 0, 0, 0, 0, cnt.data_ptr(), stream()), "scan_compact n=0")
    torch.cuda.synchronize()
    assert int(cnt.item()) == 0


def test_in_place_and_misaligned():
    a = data(9 * 16384 + 321, 4400, np.int32)
    check(a, "nonzero", inplace=True)
    for mis in (1, 2, 3):
        check(a, "nonzero", misalign=mis)


def test_full_size():
    a = data(1 << 28, 4500, np.int32, zero_frac=0.5)
    check(a, "greater", 0)
