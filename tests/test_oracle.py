"""The oracle against its pins (no GPU), plus planted mistakes that the pins
must catch.  Every mutant is a copy of the oracle with one plausible error."""
import numpy as np
import pytest

import oracle
import pins


def _int(a, ex, rev):
    return oracle.scan_int(a, exclusive=ex, reverse=rev)


def _int_out(a, ex, rev, out):
    return oracle.scan_int(a, exclusive=ex, reverse=rev, out=out)


def _seg(a, off, ex, rev):
    return oracle.segmented_int(a, off, exclusive=ex, reverse=rev)


def _f(a, ex, rev):
    return oracle.scan_f32(a, exclusive=ex, reverse=rev)


def _segf(a, off, ex, rev):
    return oracle.segmented_f32(a, off, exclusive=ex, reverse=rev)


def test_oracle_int_flat_pinned():
    assert pins.pin_int_flat(_int) == []


def test_oracle_int_inplace_pinned():
    assert pins.pin_int_inplace(_int_out) == []


def test_oracle_int_segmented_pinned():
    assert pins.pin_int_segmented(_seg) == []


def test_oracle_f32_pinned():
    assert pins.pin_f32(_f) == []


def test_oracle_f32_segmented_pinned():
    assert pins.pin_f32_segmented(_segf) == []


def test_oracle_operators_pinned():
    assert pins.pin_int_operators(lambda a, op, ex, rev: oracle.scan_op(a, op, ex, rev)) == []


def test_oracle_operators_segmented_pinned():
    assert pins.pin_int_operators_segmented(
        lambda a, off, op, ex, rev: oracle.segmented_op(a, off, op, ex, rev)) == []


def test_oracle_compact_pinned():
    assert pins.pin_compact(lambda a, p, t: oracle.compact(a, p, t)) == []


def _m_compact_keep_ge(a, p, t):
    a = np.asarray(a)
    if p == "greater":
        return a[a >= np.array(t, dtype=a.dtype)]
    return oracle.compact(a, p, t)


def _m_compact_unsigned(a, p, t):
    a = np.asarray(a)
    if p == "greater" and a.dtype == np.int32:
        return oracle.compact(a.view(np.uint32), p, np.array(t, dtype=np.int32).view(np.uint32)).view(np.int32)
    return oracle.compact(a, p, t)


def _m_compact_unordered(a, p, t):
    return np.sort(np.asarray(oracle.compact(a, p, t)))


@pytest.mark.parametrize("mutant", [_m_compact_keep_ge, _m_compact_unsigned, _m_compact_unordered])
def test_pins_catch_compact_mutant(mutant):
    assert pins.pin_compact(mutant) != []


def test_tolerance_scale():
    s, ab = oracle.scan_f32(np.array([1.0, -3.0], dtype=np.float32))
    assert np.array_equal(oracle.f32_tolerance(ab), np.array([1.0, 4.0]) * 2.0**-20)


def test_offsets_validation():
    a = np.zeros(4, dtype=np.int32)
    with pytest.raises(ValueError):
        oracle.segmented_int(a, np.array([1, 4]))
    with pytest.raises(ValueError):
        oracle.segmented_int(a, np.array([0, 3]))
    with pytest.raises(ValueError):
        oracle.segmented_int(a, np.array([0, 3, 2, 4]))


# ------------------------------------------------------------ planted mistakes

def _m_exclusive_is_inclusive(a, ex, rev):
    return oracle.scan_int(a, exclusive=False, reverse=rev)


def _m_dropped_first_term(a, ex, rev):
    out = np.asarray(oracle.scan_int(a, exclusive=ex, reverse=rev)).view(np.uint32).copy()
    if out.size and not rev:
        first = np.asarray(a).view(np.uint32)[0]
        out[1:] -= first  # a[0] missing from every later prefix
    return out


def _m_reverse_ignored(a, ex, rev):
    return oracle.scan_int(a, exclusive=ex, reverse=False)


def _m_saturating(a, ex, rev):
    v = np.asarray(a).view(np.uint32).astype(np.int64)
    if rev:
        v = v[::-1]
    c = np.cumsum(v) - (v if ex else 0)
    c = np.minimum(c, 2**32 - 1)  # no wrap-around
    return (c[::-1] if rev else c).astype(np.uint32)


def _m_off_by_one_shift(a, ex, rev):
    out = np.asarray(oracle.scan_int(a, exclusive=ex, reverse=rev)).view(np.uint32)
    return np.roll(out, 1)


def _m_seg_no_restart_after_empty(a, off, ex, rev):
    # drops empty segments' boundaries AND merges the segment after an empty one
    off = np.asarray(off)
    keep = [0]
    for s in range(1, len(off)):
        if off[s] != off[s - 1] or s == len(off) - 1:
            keep.append(s)
        else:
            keep.pop() if len(keep) > 1 else None
    return oracle.segmented_int(a, off[np.array(sorted(set(keep)))], exclusive=ex, reverse=rev)


def _m_seg_restart_late(a, off, ex, rev):
    off = np.asarray(off).copy()
    n = int(off[-1])
    off[1:-1] = np.minimum(off[1:-1] + 1, n)
    off = np.maximum.accumulate(off)
    return oracle.segmented_int(a, off, exclusive=ex, reverse=rev)


def _m_f32_accumulator(a, ex, rev):
    v = np.asarray(a, dtype=np.float32)
    if rev:
        v = v[::-1]
    c = np.cumsum(v, dtype=np.float32).astype(np.float64)
    if ex:
        c = c - v
    ab = np.cumsum(np.abs(v).astype(np.float64)) - (np.abs(v) if ex else 0)
    return (c[::-1], ab[::-1]) if rev else (c, ab)


def _m_abs_signed(a, ex, rev):
    s, _ = oracle.scan_f32(a, exclusive=ex, reverse=rev)
    return s, s.copy()


@pytest.mark.parametrize("mutant", [
    _m_exclusive_is_inclusive, _m_dropped_first_term, _m_reverse_ignored,
    _m_saturating, _m_off_by_one_shift])
def test_pins_catch_int_mutant(mutant):
    assert pins.pin_int_flat(mutant) != []


@pytest.mark.parametrize("mutant", [_m_seg_no_restart_after_empty, _m_seg_restart_late])
def test_pins_catch_segmented_mutant(mutant):
    assert pins.pin_int_segmented(mutant) != []


@pytest.mark.parametrize("mutant", [_m_f32_accumulator, _m_abs_signed])
def test_pins_catch_f32_mutant(mutant):
    assert pins.pin_f32(mutant) != []


# planted mistakes in the operator oracle
def _m_op_unsigned_compare(a, op, ex, rev):
    return oracle.scan_op(np.asarray(a).view(np.uint32), op, ex, rev).view(np.asarray(a).dtype)


def _m_op_zero_identity(a, op, ex, rev):
    out = np.asarray(oracle.scan_op(a, op, ex, rev)).copy()
    if ex and out.size:
        out[-1 if rev else 0] = 0
    return out


def _m_op_exclusive_is_inclusive(a, op, ex, rev):
    return oracle.scan_op(a, op, False, rev)


def _m_op_or_for_xor(a, op, ex, rev):
    if op != "xor":
        return oracle.scan_op(a, op, ex, rev)
    v = np.asarray(a).view(np.uint32)
    v = v[::-1] if rev else v
    out = np.bitwise_or.accumulate(v) if v.size else v
    if ex:
        out = np.concatenate([[0], out[:-1]]).astype(np.uint32)
    return (out[::-1] if rev else out).view(np.asarray(a).dtype)


def _m_op_reverse_ignored(a, op, ex, rev):
    return oracle.scan_op(a, op, ex, False)


@pytest.mark.parametrize("mutant", [_m_op_unsigned_compare, _m_op_zero_identity, _m_op_exclusive_is_inclusive,
                                    _m_op_or_for_xor, _m_op_reverse_ignored])
def test_pins_catch_operator_mutant(mutant):
    assert pins.pin_int_operators(mutant) != []


# ---------------------------------------------------------------- 64-bit integers

def test_oracle_int64_pinned():
    assert pins.pin_int64(lambda a, ex, rev: oracle.scan_int64(a, exclusive=ex, reverse=rev)) == []


def _m64_split_halves(a, ex, rev):
    # scans the two 32-bit halves separately: the carry out of the low half is lost
    v = np.ascontiguousarray(a).view(np.uint64)
    lo = np.asarray(oracle.scan_int((v & np.uint64(0xFFFFFFFF)).astype(np.uint32), exclusive=ex,
                                    reverse=rev)).astype(np.uint64)
    hi = np.asarray(oracle.scan_int((v >> np.uint64(32)).astype(np.uint32), exclusive=ex,
                                    reverse=rev)).astype(np.uint64)
    return ((hi << np.uint64(32)) | lo).view(np.asarray(a).dtype)


def _m64_float_accumulator(a, ex, rev):
    v = np.ascontiguousarray(a).view(np.uint64).astype(np.float64)
    c = np.cumsum(v) - (v if ex else 0)
    return np.mod(c, 2.0**64).astype(np.uint64).view(np.asarray(a).dtype)


def _m64_exclusive_is_inclusive(a, ex, rev):
    return oracle.scan_int64(a, exclusive=False, reverse=rev)


def _m64_reverse_ignored(a, ex, rev):
    return oracle.scan_int64(a, exclusive=ex)


def _m64_no_wrap_signed(a, ex, rev):
    # accumulates in signed 64 bits saturating at the int64 range
    v = [int(x) for x in np.ascontiguousarray(a).view(np.int64)]
    out, acc = [], 0
    for x in v:
        if ex:
            out.append(acc)
            acc = max(min(acc + x, 2**63 - 1), -2**63)
        else:
            acc = max(min(acc + x, 2**63 - 1), -2**63)
            out.append(acc)
    return np.array(out, dtype=np.int64).view(np.asarray(a).dtype)


@pytest.mark.parametrize("mutant", [_m64_split_halves, _m64_float_accumulator, _m64_exclusive_is_inclusive,
                                    _m64_no_wrap_signed, _m64_reverse_ignored])
def test_pins_catch_int64_mutant(mutant):
    assert pins.pin_int64(mutant) != []


# ---------------------------------------------------------------- float64

def test_oracle_f64_pinned():
    assert pins.pin_f64(lambda a, ex, rev: oracle.scan_f64(a, exclusive=ex, reverse=rev)) == []


def _mf64_naive(a, ex, rev):
    # plain left-to-right float64 accumulation: loses the cancellation
    v = np.asarray(a, dtype=np.float64)
    c = np.add.accumulate(v)
    ab = np.add.accumulate(np.abs(v))
    if ex:
        c = np.concatenate([[0.0], c[:-1]])
        ab = np.concatenate([[0.0], ab[:-1]])
    return c, ab


def _mf64_f32_accumulator(a, ex, rev):
    v = np.asarray(a, dtype=np.float64)
    c = np.cumsum(v.astype(np.float32), dtype=np.float32).astype(np.float64)
    _, ab = oracle.scan_f64(a, exclusive=ex)
    if ex:
        c = np.concatenate([[0.0], c[:-1]])
    return c, ab


def _mf64_exclusive_is_inclusive(a, ex, rev):
    return oracle.scan_f64(a, exclusive=False, reverse=rev)


def _mf64_reverse_ignored(a, ex, rev):
    return oracle.scan_f64(a, exclusive=ex)


def _mf64_dropped_first(a, ex, rev):
    v = np.asarray(a, dtype=np.float64).copy()
    if v.size:
        v[0] = 0.0
    return oracle.scan_f64(v, exclusive=ex, reverse=rev)


@pytest.mark.parametrize("mutant", [_mf64_naive, _mf64_f32_accumulator, _mf64_exclusive_is_inclusive,
                                    _mf64_dropped_first, _mf64_reverse_ignored])
def test_pins_catch_f64_mutant(mutant):
    assert pins.pin_f64(mutant) != []


def test_f64_tolerance_scale():
    ab = np.array([0.0, 1.0, 2.0**40])
    t = oracle.f64_tolerance(ab, 127)
    assert t[0] == 0.0 and np.allclose(t[1:], ab[1:] * 128 * 2.0**-53, rtol=1e-5)


# ---------------------------------------------------------------- two-way partition

def test_oracle_partition_pinned():
    assert pins.pin_partition(oracle.partition) == []


def _mp_rejected_in_order(a, pred, thr):
    out, k = oracle.partition(a, pred, thr)
    out = np.asarray(out).copy()
    out[k:] = out[k:][::-1]
    return out, k


def _mp_swapped(a, pred, thr):
    out, k = oracle.partition(a, pred, thr)
    out = np.asarray(out)
    return np.concatenate([out[k:][::-1], out[:k]]), out.size - k


def _mp_off_by_one(a, pred, thr):
    out, k = oracle.partition(a, pred, thr)
    return np.roll(np.asarray(out), 1), k


@pytest.mark.parametrize("mutant", [_mp_rejected_in_order, _mp_swapped, _mp_off_by_one])
def test_pins_catch_partition_mutant(mutant):
    assert pins.pin_partition(mutant) != []


# ---------------------------------------------------------------- non-finite values

def _f64(a, ex, rev):
    return oracle.scan_f64(a, exclusive=ex, reverse=rev)


def test_oracle_f32_nonfinite_pinned():
    assert pins.pin_nonfinite(_f, np.float32) == []


def test_oracle_f32_segmented_nonfinite_pinned():
    assert pins.pin_nonfinite_segmented(_segf) == []


def test_oracle_f64_nonfinite_pinned():
    assert pins.pin_nonfinite(_f64, np.float64) == []


def _mnf_abs_skips_nan(a, ex, rev):
    # a tolerance scale that stays finite after a NaN
    s, _ = oracle.scan_f32(a, exclusive=ex, reverse=rev)
    v = np.abs(np.asarray(a, dtype=np.float64))
    v = v[::-1] if rev else v
    ab = np.nancumsum(v) - (np.nan_to_num(v, nan=0.0) if ex else 0)
    return s, (ab[::-1] if rev else ab)


def _mnf_sum_drops_nan(a, ex, rev):
    # NaN read as 0 in the running total
    a = np.asarray(a, dtype=np.float32)
    _, ab = oracle.scan_f32(a, exclusive=ex, reverse=rev)
    s, _ = oracle.scan_f32(np.where(np.isnan(a), np.float32(0), a), exclusive=ex, reverse=rev)
    return s, ab


def _mnf_inf_minus_inf_zero(a, ex, rev):
    # +inf + -inf taken as 0 instead of NaN
    s, ab = oracle.scan_f32(a, exclusive=ex, reverse=rev)
    a = np.asarray(a, dtype=np.float32)
    nan_in = np.isnan(a).any()
    if not nan_in:
        s = np.where(np.isnan(s), 0.0, s)
    return s, ab


def _mf64_unguarded_two_sum(a, ex, rev):
    # double-double accumulation whose TwoSum error term is used even when the
    # sum is infinite (inf - inf = NaN turns +inf into NaN)
    v = np.asarray(a, dtype=np.float64)
    idx = range(v.size - 1, -1, -1) if rev else range(v.size)
    s = np.empty(v.size)
    ab = np.empty(v.size)
    hi = lo = aacc = 0.0
    with np.errstate(invalid="ignore", over="ignore"):
        for i in idx:
            x = float(v[i])
            if ex:
                s[i], ab[i] = hi, aacc
            t = hi + x
            bv = t - hi
            e = ((hi - (t - bv)) + (x - bv)) + lo
            hi, lo = t + e, e - ((t + e) - t)
            aacc += abs(x)
            if not ex:
                s[i], ab[i] = hi, aacc
    return s, ab


@pytest.mark.parametrize("mutant", [_mnf_abs_skips_nan, _mnf_sum_drops_nan, _mnf_inf_minus_inf_zero])
def test_nonfinite_pins_catch_f32_mutant(mutant):
    assert pins.pin_nonfinite(mutant, np.float32) != []


def test_nonfinite_pins_catch_f64_mutant():
    assert pins.pin_nonfinite(_mf64_unguarded_two_sum, np.float64) != []


def _mnf_seg_nan_leaks(a, off, ex, rev):
    # the segment restart clears the value but not a sticky NaN state
    s, ab = oracle.segmented_f32(a, off, exclusive=ex, reverse=rev)
    flat, _ = oracle.scan_f32(a, exclusive=ex, reverse=rev)
    return np.where(np.isnan(flat), np.nan, s), ab


def test_nonfinite_pins_catch_segmented_mutant():
    assert pins.pin_nonfinite_segmented(_mnf_seg_nan_leaks) != []
