"""Pins for the sequential oracle: checks that do not use the oracle itself.

Each ``pin_*`` function takes an implementation with the oracle's call
signature and returns a list of failure strings (empty = pinned).  The real
oracle must pass them all; ``test_oracle.py`` also plants plausible mistakes
in copies of the oracle and checks that some pin catches each one.

Sources of truth (none of them is the oracle):
  * hand-computed fixtures under tests/golden/ (definition in the Introduction),
  * closed forms (constant and arithmetic-progression inputs),
  * brute force from the definition in pure Python integers / fractions,
  * numpy's own cumulative sums (uint32 wraps; float64 add.accumulate runs
    left to right),
  * invariants (last inclusive value = total, inclusive - exclusive = input,
    linearity modulo 2^32, in place = out of place).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

import golden_io

M32 = 1 << 32


def _brute_int(a, exclusive, reverse):
    """O(n^2) scan straight from the definition, in Python integers mod 2^32."""
    a = [int(x) % M32 for x in a]
    n = len(a)
    out = []
    for i in range(n):
        if not reverse:
            idx = range(0, i) if exclusive else range(0, i + 1)
        else:
            idx = range(i + 1, n) if exclusive else range(i, n)
        out.append(sum(a[j] for j in idx) % M32)
    return out


def _cmp(name, got, want, fails):
    got = [int(x) for x in np.asarray(got).view(np.uint32)] if np.asarray(got).dtype.kind in "iu" else list(got)
    want = [int(x) % M32 for x in want]
    if got != want:
        bad = next(i for i, (g, w) in enumerate(zip(got, want)) if g != w) if len(got) == len(want) else -1
        fails.append("%s: mismatch (first at %d)" % (name, bad))


# ---------------------------------------------------------------- integers

def pin_int_flat(scan_int) -> list:
    """scan_int(a, exclusive, reverse) -> array, wrapping modulo 2^32."""
    fails = []
    g = golden_io.load("definition_small.txt")
    a = np.array(g["input"], dtype=np.uint32)
    _cmp("golden inclusive", scan_int(a, False, False), g["inclusive"], fails)
    _cmp("golden exclusive", scan_int(a, True, False), g["exclusive"], fails)
    _cmp("golden reverse inclusive", scan_int(a, False, True), g["reverse_inclusive"], fails)
    _cmp("golden reverse exclusive", scan_int(a, True, True), g["reverse_exclusive"], fails)
    w = golden_io.load("wrap_u32.txt")
    a = np.array(w["input"], dtype=np.uint32)
    _cmp("golden wrap inclusive", scan_int(a, False, False), w["inclusive"], fails)
    _cmp("golden wrap exclusive", scan_int(a, True, False), w["exclusive"], fails)

    # closed form: all ones -> i+1 (inclusive), i (exclusive); reverse n-i / n-1-i
    n = 5000
    ones = np.ones(n, dtype=np.uint32)
    i = np.arange(n, dtype=np.int64)
    _cmp("ones inclusive", scan_int(ones, False, False), i + 1, fails)
    _cmp("ones exclusive", scan_int(ones, True, False), i, fails)
    _cmp("ones reverse inclusive", scan_int(ones, False, True), n - i, fails)
    _cmp("ones reverse exclusive", scan_int(ones, True, True), n - 1 - i, fails)

    # closed form: a_i = c + d*i  ->  (i+1)c + d*i(i+1)/2  (mod 2^32), chosen to wrap
    c, d = 3_000_000_007 % M32, 2_654_435_761
    n = 20000
    a = np.array([(c + d * k) % M32 for k in range(n)], dtype=np.uint32)
    want = [((k + 1) * c + d * k * (k + 1) // 2) % M32 for k in range(n)]
    _cmp("arithmetic progression inclusive", scan_int(a, False, False), want, fails)
    want_ex = [(k * c + d * (k - 1) * k // 2) % M32 for k in range(n)]
    _cmp("arithmetic progression exclusive", scan_int(a, True, False), want_ex, fails)

    # brute force from the definition on small random inputs, every mode
    rng = np.random.default_rng(7)
    for n in (0, 1, 2, 3, 17, 64, 65, 257):
        a = rng.integers(0, M32, size=n, dtype=np.uint32)
        for ex in (False, True):
            for rev in (False, True):
                _cmp("brute n=%d ex=%d rev=%d" % (n, ex, rev),
                     scan_int(a, ex, rev), _brute_int(a, ex, rev), fails)

    # numpy's wrapping uint32 cumsum (forward) and its flip (reverse)
    a = rng.integers(0, M32, size=100_003, dtype=np.uint32)
    _cmp("numpy cumsum uint32", scan_int(a, False, False), np.cumsum(a, dtype=np.uint32), fails)
    _cmp("numpy flipped cumsum", scan_int(a, False, True),
         np.cumsum(a[::-1], dtype=np.uint32)[::-1], fails)

    # invariants: last = total, inclusive - exclusive = input, linearity, in place
    inc = np.asarray(scan_int(a, False, False)).view(np.uint32)
    exc = np.asarray(scan_int(a, True, False)).view(np.uint32)
    total = int(a.astype(np.uint64).sum()) % M32
    if int(inc[-1]) != total:
        fails.append("last inclusive != total")
    if not np.array_equal(inc - exc, a):
        fails.append("inclusive - exclusive != input")
    b = rng.integers(0, M32, size=a.size, dtype=np.uint32)
    lin = np.asarray(scan_int(a + b, False, False)).view(np.uint32)
    if not np.array_equal(lin, inc + np.asarray(scan_int(b, False, False)).view(np.uint32)):
        fails.append("scan(a+b) != scan(a)+scan(b) mod 2^32")
    # signed view: int32 input gives the same bits as uint32
    s = np.asarray(scan_int(a.view(np.int32), False, False))
    if s.dtype != np.int32 or not np.array_equal(s.view(np.uint32), inc):
        fails.append("int32 view differs from uint32")
    return fails


M64 = 1 << 64


def _cmp64(name, got, want, fails):
    got = [int(x) for x in np.asarray(got).view(np.uint64)]
    want = [int(x) % M64 for x in want]
    if got != want:
        bad = next(i for i, (g, w) in enumerate(zip(got, want)) if g != w) if len(got) == len(want) else -1
        fails.append("%s: mismatch (first at %d)" % (name, bad))


def pin_int64(scan64) -> list:
    """scan64(a, exclusive, reverse) -> array: scan wrapping modulo 2^64."""
    fails = []
    g = golden_io.load("wrap_u64.txt")
    a = np.array(g["input"], dtype=np.uint64)
    _cmp64("golden inclusive", scan64(a, False, False), g["inclusive"], fails)
    _cmp64("golden exclusive", scan64(a, True, False), g["exclusive"], fails)
    _cmp64("golden reverse inclusive", scan64(a, False, True), g["reverse_inclusive"], fails)
    _cmp64("golden reverse exclusive", scan64(a, True, True), g["reverse_exclusive"], fails)

    # closed form: a_i = c + d*i (mod 2^64) -> (i+1)c + d*i(i+1)/2, with values
    # that carry out of the low 32 bits at every step and wrap past 2^64
    c, d = 0xFFFFFFFF, 0x9E3779B97F4A7C15
    n = 20000
    a = np.array([(c + d * k) % M64 for k in range(n)], dtype=np.uint64)
    want = [((k + 1) * c + d * k * (k + 1) // 2) % M64 for k in range(n)]
    _cmp64("arithmetic progression inclusive", scan64(a, False, False), want, fails)
    want_ex = [(k * c + d * (k - 1) * k // 2) % M64 for k in range(n)]
    _cmp64("arithmetic progression exclusive", scan64(a, True, False), want_ex, fails)

    # brute force from the definition in Python integers
    rng = np.random.default_rng(11)
    for n in (0, 1, 2, 3, 17, 64, 65, 257):
        a = rng.integers(0, M64, size=n, dtype=np.uint64)
        v = [int(x) for x in a]
        for ex in (False, True):
            want = [sum(v[:i] if ex else v[:i + 1]) for i in range(n)]
            _cmp64("brute n=%d ex=%d" % (n, ex), scan64(a, ex, False), want, fails)
            want = [sum(v[i + 1:] if ex else v[i:]) for i in range(n)]
            _cmp64("brute reverse n=%d ex=%d" % (n, ex), scan64(a, ex, True), want, fails)

    # numpy's wrapping uint64 cumsum
    a = rng.integers(0, M64, size=100_003, dtype=np.uint64)
    inc = np.asarray(scan64(a, False, False)).view(np.uint64)
    exc = np.asarray(scan64(a, True, False)).view(np.uint64)
    if not np.array_equal(inc, np.cumsum(a, dtype=np.uint64)):
        fails.append("numpy cumsum uint64")
    if not np.array_equal(np.asarray(scan64(a, False, True)).view(np.uint64),
                          np.cumsum(a[::-1], dtype=np.uint64)[::-1]):
        fails.append("numpy flipped cumsum uint64")
    # invariants: inclusive - exclusive = input; the low 32 bits are the
    # 32-bit scan of the low halves
    if not np.array_equal(inc - exc, a):
        fails.append("inclusive - exclusive != input")
    lo = (a & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    if not np.array_equal((inc & np.uint64(0xFFFFFFFF)).astype(np.uint32), np.cumsum(lo, dtype=np.uint32)):
        fails.append("low halves differ from the 32-bit scan")
    # signed view: negative int64 input, the same bits as uint64
    neg = -np.arange(1, 1001, dtype=np.int64)
    s = np.asarray(scan64(neg, False, False))
    if s.dtype != np.int64 or [int(x) for x in s] != [-(k + 1) * (k + 2) // 2 for k in range(1000)]:
        fails.append("int64 negative input")
    return fails


def pin_f64(scan_f64) -> list:
    """scan_f64(a, exclusive, reverse) -> (sums float64, abs_sums float64):
    the exact prefix (reverse: suffix) sums rounded to float64."""
    fails = []
    g = golden_io.load("cancel_f64.txt", conv=float)
    a = np.array(g["input"], dtype=np.float64)
    for key, ex, rev in (("inclusive", False, False), ("exclusive", True, False),
                         ("reverse_inclusive", False, True), ("reverse_exclusive", True, True)):
        s, _ = scan_f64(a, ex, rev)
        _fcmp("golden cancel " + key, s, g[key], fails)

    # closed form: a_i = i (integers below 2^26: every partial sum exact)
    n = 60_000
    a = np.arange(n, dtype=np.float64)
    k = np.arange(n, dtype=np.int64)
    s, ab = scan_f64(a, False, False)
    _fcmp("arithmetic progression inclusive", s, k * (k + 1) // 2, fails)
    _fcmp("abs of a nonnegative input", ab, k * (k + 1) // 2, fails)
    s, _ = scan_f64(a, True, False)
    _fcmp("arithmetic progression exclusive", s, (k - 1) * k // 2, fails)
    s, _ = scan_f64(a, False, True)
    tot = (n - 1) * n // 2
    _fcmp("arithmetic progression reverse", s, tot - (k - 1) * k // 2, fails)

    # exact rational prefix sums, rounded once, over a wide exponent range
    rng = np.random.default_rng(19)
    a = rng.standard_normal(400) * np.ldexp(1.0, rng.integers(-30, 30, size=400))
    s, ab = scan_f64(a, False, False)
    acc = Fraction(0)
    for i, x in enumerate(a):
        acc += Fraction(float(x))
        ulp = Fraction(math.ulp(float(acc))) if acc != 0 else Fraction(0)
        # correctly rounded up to the tiny double-double error
        if abs(Fraction(float(s[i])) - acc) > ulp / 2 + Fraction(2.0**-100) * Fraction(float(ab[i])):
            fails.append("rational exact sum at %d" % i)
            break
    # math.fsum (correctly rounded sum of floats) at sampled prefixes
    a = rng.standard_normal(200_001) * 1e3
    s, ab = scan_f64(a, False, False)
    for i in list(range(0, a.size, 9_973)) + [a.size - 1]:
        want = math.fsum(a[:i + 1].tolist())
        if abs(float(s[i]) - want) > math.ulp(want) / 2 + 2.0**-95 * float(ab[i]):
            fails.append("fsum prefix at %d" % i)
            break
    r, rab = scan_f64(a, False, True)
    for i in [0] + list(range(7, a.size, 11_113)):
        want = math.fsum(a[i:].tolist())
        if abs(float(r[i]) - want) > math.ulp(want) / 2 + 2.0**-95 * float(rab[i]):
            fails.append("fsum suffix at %d" % i)
            break
    # exclusive is the inclusive result shifted by one, identity first
    e, eab = scan_f64(a, True, False)
    if e[0] != 0.0 or not np.array_equal(e[1:], s[:-1]):
        fails.append("exclusive != shifted inclusive")
    if abs(float(ab[-1]) - math.fsum(np.abs(a).tolist())) > a.size * 2.0**-53 * float(ab[-1]):
        fails.append("abs sum total")
    return fails


def pin_partition(partition) -> list:
    """partition(a, predicate, threshold) -> (out, k): kept elements first in
    order, the rest after them in reverse order."""
    fails = []
    g = golden_io.load("partition_small.txt")
    a = np.array(g["input"], dtype=np.int32)
    rej = [0 if x != 0 else 1 for x in g["input"]]
    if [sum(rej[:i]) for i in range(len(rej))] != g["rejected_positions"]:
        fails.append("fixture rejection positions are not the exclusive scan of the rejections")
    out, k = partition(a, "nonzero", 0)
    _cmp("golden nonzero", out, g["nonzero_out"], fails)
    if k != g["nonzero_kept_count"][0]:
        fails.append("golden nonzero count")
    out, k = partition(a, "greater", 2)
    _cmp("golden > 2", out, g["greater_2_out"], fails)
    if k != g["greater_2_kept_count"][0]:
        fails.append("golden > 2 count")
    # numpy masks: kept part in order, rejected part reversed, for every dtype
    rng = np.random.default_rng(91)
    for dt in (np.int32, np.uint32):
        x = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=7001, dtype=np.int64, endpoint=True).astype(dt)
        x[rng.random(x.size) < 0.4] = 0
        thr = dt(rng.integers(np.iinfo(dt).min // 2, np.iinfo(dt).max // 2))
        for pred, keep in (("nonzero", x != 0), ("greater", x > thr)):
            out, k = partition(x, pred, thr if pred == "greater" else 0)
            want = np.concatenate([x[keep], x[~keep][::-1]])
            if k != int(keep.sum()) or not np.array_equal(np.asarray(out).view(np.uint32), want.view(np.uint32)):
                fails.append("numpy mask %s %s" % (pred, np.dtype(dt).name))
    f = rng.standard_normal(3001).astype(np.float32)
    f[::89] = np.nan
    keep = f > np.float32(-0.5)
    out, k = partition(f, "greater", np.float32(-0.5))
    want = np.concatenate([f[keep], f[~keep][::-1]])
    if k != int(keep.sum()) or not np.array_equal(np.asarray(out).view(np.uint32), want.view(np.uint32)):
        fails.append("numpy mask float32 (NaN rejected)")
    # special cases: nothing kept (the input reversed), everything kept (a
    # copy), empty input
    o = np.arange(1, 101, dtype=np.int32)
    out, k = partition(o, "greater", 1000)
    if k != 0 or not np.array_equal(out, o[::-1]):
        fails.append("nothing kept = reversed input")
    out, k = partition(o, "greater", 0)
    if k != 100 or not np.array_equal(out, o):
        fails.append("everything kept = copy")
    out, k = partition(np.zeros(0, dtype=np.int32), "nonzero", 0)
    if k != 0 or np.asarray(out).size != 0:
        fails.append("empty input")
    return fails


def pin_int_inplace(scan_int_out) -> list:
    """scan_int_out(a, exclusive, reverse, out) with out == a."""
    fails = []
    rng = np.random.default_rng(11)
    for ex in (False, True):
        for rev in (False, True):
            a = rng.integers(0, M32, size=4099, dtype=np.uint32)
            want = _brute_int(a[:300], ex, rev) if not rev else None
            ref = np.cumsum(a, dtype=np.uint32) if not rev else np.cumsum(a[::-1], dtype=np.uint32)[::-1]
            if ex:
                ref = (ref - a).astype(np.uint32)
            buf = a.copy()
            scan_int_out(buf, ex, rev, buf)
            if not np.array_equal(buf, ref):
                fails.append("in place ex=%d rev=%d" % (ex, rev))
            if want is not None and [int(x) for x in buf[:300]] != want:
                fails.append("in place brute ex=%d" % ex)
    return fails


def pin_int_segmented(seg_int, scan_int_brute=_brute_int) -> list:
    """seg_int(a, offsets, exclusive, reverse) -> array."""
    fails = []
    g = golden_io.load("segmented_small.txt")
    a = np.array(g["input"], dtype=np.uint32)
    off = np.array(g["offsets"], dtype=np.int64)
    _cmp("golden seg inclusive", seg_int(a, off, False, False), g["inclusive"], fails)
    _cmp("golden seg exclusive", seg_int(a, off, True, False), g["exclusive"], fails)
    _cmp("golden seg reverse inclusive", seg_int(a, off, False, True), g["reverse_inclusive"], fails)

    rng = np.random.default_rng(13)
    for n, S in ((1, 1), (50, 1), (50, 7), (400, 40), (300, 300), (257, 90)):
        a = rng.integers(0, M32, size=n, dtype=np.uint32)
        if S == 1:
            off = np.array([0, n], dtype=np.int64)
        else:
            cuts = np.sort(rng.integers(0, n + 1, size=S - 1))
            off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
        for ex in (False, True):
            for rev in (False, True):
                want = []
                for s in range(S):
                    want += scan_int_brute(a[off[s]:off[s + 1]], ex, rev)
                _cmp("seg brute n=%d S=%d ex=%d rev=%d" % (n, S, ex, rev),
                     seg_int(a, off, ex, rev), want, fails)
    # all length-1 segments: inclusive = input, exclusive = 0
    n = 1000
    a = rng.integers(0, M32, size=n, dtype=np.uint32)
    off = np.arange(n + 1, dtype=np.int64)
    _cmp("length-1 inclusive", seg_int(a, off, False, False), a, fails)
    _cmp("length-1 exclusive", seg_int(a, off, True, False), np.zeros(n, dtype=np.int64), fails)
    # a single segment is the flat scan (numpy wrapping cumsum)
    a = rng.integers(0, M32, size=10_000, dtype=np.uint32)
    _cmp("single segment = flat", seg_int(a, np.array([0, a.size]), False, False),
         np.cumsum(a, dtype=np.uint32), fails)
    return fails


# ---------------------------------------------------------------- floats

def _fcmp(name, got, want, fails, exact=True, tol=None):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if got.shape != want.shape:
        fails.append("%s: shape %s vs %s" % (name, got.shape, want.shape))
        return
    if exact:
        if not np.array_equal(got, want):
            fails.append("%s: not bit-equal (first at %d)" % (name, int(np.argmax(got != want))))
    else:
        err = np.abs(got - want)
        if np.any(err > tol):
            fails.append("%s: error %.3g above bound at %d" % (name, float(err.max()), int(np.argmax(err > tol))))


def pin_f32(scan_f32) -> list:
    """scan_f32(a, exclusive, reverse) -> (sums float64, abs_sums float64)."""
    fails = []
    g = golden_io.load("float_small.txt", conv=float)
    a = np.array(g["input"], dtype=np.float32)
    s, ab = scan_f32(a, False, False)
    _fcmp("golden f inclusive", s, g["inclusive"], fails)
    _fcmp("golden f abs", ab, g["abs_inclusive"], fails)
    s, _ = scan_f32(a, True, False)
    _fcmp("golden f exclusive", s, g["exclusive"], fails)

    rng = np.random.default_rng(17)
    # integer-valued inputs: every partial sum exact -> integer cumsum
    a = rng.integers(-1000, 1001, size=50_000).astype(np.float32)
    ai = a.astype(np.int64)
    for ex in (False, True):
        for rev in (False, True):
            v = ai[::-1] if rev else ai
            ref = np.cumsum(v)
            if ex:
                ref = ref - v
            if rev:
                ref = ref[::-1]
            s, ab = scan_f32(a, ex, rev)
            _fcmp("int-valued ex=%d rev=%d" % (ex, rev), s, ref, fails)
            vabs = np.abs(v)
            rab = np.cumsum(vabs) - (vabs if ex else 0)
            _fcmp("abs int-valued ex=%d rev=%d" % (ex, rev), ab, rab[::-1] if rev else rab, fails)

    # numpy's float64 add.accumulate runs left to right: bit-equal
    a = rng.standard_normal(100_001).astype(np.float32)
    s, _ = scan_f32(a, False, False)
    _fcmp("numpy add.accumulate f64", s, np.add.accumulate(a.astype(np.float64)), fails)
    s, _ = scan_f32(a, False, True)
    _fcmp("numpy flipped accumulate f64", s, np.add.accumulate(a[::-1].astype(np.float64))[::-1], fails)

    # exact rational prefix sums on a small random input: the sequential float64
    # sum is within (i) * 2^-53 * sum|a| of the exact value (standard bound)
    a = rng.standard_normal(600).astype(np.float32)
    s, ab = scan_f32(a, False, False)
    exact = []
    acc = Fraction(0)
    for x in a:
        acc += Fraction(float(x))
        exact.append(acc)
    for k in range(len(a)):
        bound = (k + 1) * 2.0**-53 * float(ab[k]) * 1.0000001
        if abs(Fraction(float(s[k])) - exact[k]) > Fraction(bound):
            fails.append("rational bound at %d" % k)
            break
    if abs(float(s[-1]) - math.fsum(float(x) for x in a)) > len(a) * 2.0**-53 * float(ab[-1]):
        fails.append("fsum total")
    return fails


def pin_f32_segmented(seg_f32) -> list:
    fails = []
    rng = np.random.default_rng(19)
    n = 3000
    a = rng.integers(-50, 51, size=n).astype(np.float32)
    cuts = np.sort(rng.integers(0, n + 1, size=39))
    off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    for ex in (False, True):
        for rev in (False, True):
            want = []
            for s in range(len(off) - 1):
                seg = a[off[s]:off[s + 1]].astype(np.int64)
                v = seg[::-1] if rev else seg
                c = np.cumsum(v) - (v if ex else 0)
                want.append(c[::-1] if rev else c)
            s, _ = seg_f32(a, off, ex, rev)
            _fcmp("seg f ex=%d rev=%d" % (ex, rev), s, np.concatenate(want), fails)
    return fails


# ---------------------------------------------------------------- non-finite values
# Reading of the definition for IEEE inputs: every output is a sum of its
# prefix (suffix for reverse scans), so its class follows from the terms it
# contains -- NaN if one of them is NaN or both infinities occur, +inf / -inf
# if only that infinity occurs, finite otherwise (finite overflow aside).
# These classes are worked out here term by term in plain Python, apart from
# the oracle's arithmetic; zeros of either sign compare equal.

def _same_float(got, want) -> bool:
    g = np.asarray(got, dtype=np.float64)
    w = np.asarray(want, dtype=np.float64)
    if g.shape != w.shape:
        return False
    return bool(np.all(np.where(np.isnan(w), np.isnan(g), g == w)))


FINITE, POS_INF, NEG_INF, NAN = 0, 1, 2, 3


def _prefix_classes(v) -> np.ndarray:
    """Class of each inclusive prefix sum of v, term by term."""
    out = np.empty(len(v), dtype=np.int8)
    pos = neg = nan = False
    for i, x in enumerate(v):
        x = float(x)
        if x != x:
            nan = True
        elif x == math.inf:
            pos = True
        elif x == -math.inf:
            neg = True
        out[i] = NAN if nan or (pos and neg) else (POS_INF if pos else (NEG_INF if neg else FINITE))
    return out


def _scan_classes(v, exclusive, reverse) -> np.ndarray:
    w = v[::-1] if reverse else v
    c = _prefix_classes(w)
    if exclusive and c.size:
        c = np.concatenate([[FINITE], c[:-1]]).astype(np.int8)
    return c[::-1] if reverse else c


def _class_of(s) -> np.ndarray:
    s = np.asarray(s, dtype=np.float64)
    return np.where(np.isnan(s), NAN, np.where(s == np.inf, POS_INF,
                    np.where(s == -np.inf, NEG_INF, FINITE))).astype(np.int8)


def _inject_nonfinite(rng, v):
    """v with 0-3 NaN / +inf / -inf planted at random positions."""
    kinds = rng.choice([np.nan, np.inf, -np.inf], size=int(rng.integers(0, 4)))
    v = v.copy()
    v[rng.integers(0, v.size, size=kinds.size)] = kinds
    return v


def pin_nonfinite(scan_f, dtype) -> list:
    """scan_f(a, exclusive, reverse) -> (sums float64, abs_sums float64) for
    float input of `dtype` (float32 or float64)."""
    fails = []
    g = golden_io.load("nonfinite.txt", conv=float)
    modes = (("inclusive", False, False), ("exclusive", True, False),
             ("reverse_inclusive", False, True), ("reverse_exclusive", True, True))
    for case in ("inf", "nan", "zero", "mix"):
        a = np.array(g[case + "_input"], dtype=dtype)
        for key, ex, rev in modes:
            if case + "_" + key in g and not _same_float(scan_f(a, ex, rev)[0], g[case + "_" + key]):
                fails.append("golden %s_%s" % (case, key))
        for key, ex in (("abs_inclusive", False), ("abs_exclusive", True)):
            if case + "_" + key in g and not _same_float(scan_f(a, ex, False)[1], g[case + "_" + key]):
                fails.append("golden %s_%s" % (case, key))

    # classes term by term on random inputs with planted NaN / infinities;
    # where every term is finite the value is the sequential sum of those
    # terms (bit-equal for float32 input summed in float64, within the
    # recursive-summation bound for the float64 reference)
    rng = np.random.default_rng(23)
    for trial in range(24):
        n = int(rng.integers(1, 3000))
        v = _inject_nonfinite(rng, rng.standard_normal(n).astype(dtype))
        for ex in (False, True):
            for rev in (False, True):
                s, ab = scan_f(v, ex, rev)
                if not np.array_equal(_class_of(s), _scan_classes(v, ex, rev)):
                    fails.append("classes trial %d ex=%d rev=%d" % (trial, ex, rev))
                if not np.array_equal(_class_of(ab), _scan_classes(np.abs(v), ex, rev)):
                    fails.append("abs classes trial %d ex=%d rev=%d" % (trial, ex, rev))
                w = (v[::-1] if rev else v).astype(np.float64)
                with np.errstate(invalid="ignore"):
                    part = np.add.accumulate(w)
                fin = np.isfinite(part)            # prefixes of finite terms only
                seq = np.where(fin, part, 0.0)
                scale = np.add.accumulate(np.where(fin, np.abs(w), 0.0))
                if ex:
                    seq, scale = np.concatenate([[0.0], seq[:-1]]), np.concatenate([[0.0], scale[:-1]])
                    fin = np.concatenate([[True], fin[:-1]])
                if rev:
                    seq, scale, fin = seq[::-1], scale[::-1], fin[::-1]
                tol = 0.0 if dtype == np.float32 else (n + 1) * 2.0**-53 * scale
                with np.errstate(invalid="ignore"):
                    bad = fin & ~(np.abs(np.asarray(s, dtype=np.float64) - seq) <= tol)
                if np.any(bad):
                    fails.append("finite values trial %d ex=%d rev=%d" % (trial, ex, rev))
    return fails


def pin_nonfinite_segmented(seg_f) -> list:
    """seg_f(a, offsets, exclusive, reverse) -> (sums, abs_sums) for float32
    input: the classes restart with every segment."""
    fails = []
    rng = np.random.default_rng(29)
    for trial in range(12):
        n = int(rng.integers(1, 4000))
        v = _inject_nonfinite(rng, rng.standard_normal(n).astype(np.float32))
        cuts = np.sort(rng.integers(0, n + 1, size=int(rng.integers(0, 30))))
        off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
        for ex in (False, True):
            for rev in (False, True):
                want = np.concatenate([_scan_classes(v[off[s]:off[s + 1]], ex, rev)
                                       for s in range(off.size - 1)])
                s, _ = seg_f(v, off, ex, rev)
                if not np.array_equal(_class_of(s), want):
                    fails.append("segmented classes trial %d ex=%d rev=%d" % (trial, ex, rev))
    return fails


# ---------------------------------------------------------------- other operators

_IDENT = {("max", True): -(1 << 31), ("max", False): 0,
          ("min", True): (1 << 31) - 1, ("min", False): M32 - 1, ("xor", True): 0, ("xor", False): 0}


def _brute_op(a, op, exclusive, reverse):
    """O(n^2) scan from the definition in Python integers: the reduction of
    each prefix (suffix for reverse), starting from the operator's identity;
    int32 compares as signed, uint32 as unsigned."""
    sgn = np.asarray(a).dtype == np.int32
    vals = [int(x) for x in a]
    n = len(vals)
    out = []
    for i in range(n):
        if not reverse:
            idx = range(0, i) if exclusive else range(0, i + 1)
        else:
            idx = range(i + 1, n) if exclusive else range(i, n)
        acc = _IDENT[(op, sgn)]
        for j in idx:
            x = vals[j]
            acc = max(acc, x) if op == "max" else min(acc, x) if op == "min" else (acc ^ x)
        out.append(acc)
    return out


def pin_int_operators(scan_op) -> list:
    """scan_op(a, op, exclusive, reverse) for op in max / min / xor."""
    fails = []
    g = golden_io.load("operators_small.txt")
    a = np.array(g["input"], dtype=np.int32)
    for key, op, ex, rev in (("max_inclusive", "max", False, False), ("max_exclusive", "max", True, False),
                             ("min_inclusive", "min", False, False), ("min_exclusive", "min", True, False),
                             ("max_reverse", "max", False, True), ("xor_inclusive", "xor", False, False),
                             ("xor_exclusive", "xor", True, False)):
        _cmp("golden " + key, scan_op(a, op, ex, rev), g[key], fails)
    u = a.view(np.uint32)
    _cmp("golden umax_inclusive", scan_op(u, "max", False, False), g["umax_inclusive"], fails)
    _cmp("golden umin_inclusive", scan_op(u, "min", False, False), g["umin_inclusive"], fails)

    # brute force from the definition, both signednesses, every form
    rng = np.random.default_rng(77)
    for dt in (np.int32, np.uint32):
        for n in (1, 2, 9, 40):
            x = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=n, dtype=np.int64, endpoint=True).astype(dt)
            for op in ("max", "min", "xor"):
                for ex in (False, True):
                    for rev in (False, True):
                        _cmp("brute %s %s n=%d ex=%d rev=%d" % (op, np.dtype(dt).name, n, ex, rev),
                             scan_op(x, op, ex, rev), _brute_op(x, op, ex, rev), fails)

    # numpy's own cumulative reductions (signed compare for int32, unsigned for uint32)
    for dt in (np.int32, np.uint32):
        x = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=20000, dtype=np.int64, endpoint=True).astype(dt)
        for op, uf in (("max", np.maximum), ("min", np.minimum), ("xor", np.bitwise_xor)):
            _cmp("numpy %s.accumulate %s" % (op, np.dtype(dt).name), scan_op(x, op, False, False),
                 uf.accumulate(x), fails)
            _cmp("numpy reversed %s %s" % (op, np.dtype(dt).name), scan_op(x, op, False, True),
                 uf.accumulate(x[::-1])[::-1], fails)

    # invariants and special cases
    x = rng.integers(-1000, 1000, size=5000).astype(np.int32)
    inc = np.asarray(scan_op(x, "xor", False, False))
    if not np.array_equal(np.bitwise_xor(inc[1:], inc[:-1]), x[1:]):
        fails.append("xor: consecutive inclusive values must differ by the input")
    for op in ("max", "min", "xor"):
        inc = np.asarray(scan_op(x, op, False, False))
        exc = np.asarray(scan_op(x, op, True, False))
        if exc[0] != _IDENT[(op, True)] or not np.array_equal(exc[1:], inc[:-1]):
            fails.append("%s: exclusive must be the identity then the inclusive shifted" % op)
    srt = np.sort(x)
    _cmp("max of ascending input = input", scan_op(srt, "max", False, False), srt, fails)
    _cmp("min of ascending input = first", scan_op(srt, "min", False, False), [int(srt[0])] * srt.size, fails)
    c = np.full(17, -5, dtype=np.int32)
    _cmp("max of a constant", scan_op(c, "max", False, False), c, fails)
    return fails


def pin_int_operators_segmented(seg_op) -> list:
    """seg_op(a, offsets, op, exclusive, reverse): per-segment scans from the
    definition, empty segments included; one segment = the flat scan."""
    fails = []
    rng = np.random.default_rng(78)
    a = rng.integers(-50, 50, size=30).astype(np.int32)
    off = np.array([0, 0, 4, 5, 5, 13, 29, 30], dtype=np.int64)
    for op in ("max", "min", "xor"):
        for ex in (False, True):
            for rev in (False, True):
                want = []
                for s in range(off.size - 1):
                    want += _brute_op(a[off[s]:off[s + 1]], op, ex, rev)
                _cmp("segmented brute %s ex=%d rev=%d" % (op, ex, rev), seg_op(a, off, op, ex, rev), want, fails)
    x = rng.integers(0, 1 << 20, size=3000).astype(np.uint32)
    _cmp("one segment = numpy max.accumulate", seg_op(x, np.array([0, x.size]), "max", False, False),
         np.maximum.accumulate(x), fails)
    return fails


# ---------------------------------------------------------------- stream compaction

def pin_compact(compact) -> list:
    """compact(a, predicate, threshold) -> kept elements in order."""
    fails = []
    g = golden_io.load("compact_small.txt")
    a = np.array(g["input"], dtype=np.int32)
    _cmp("golden nonzero", compact(a, "nonzero", 0), g["nonzero_kept"], fails)
    _cmp("golden > 2", compact(a, "greater", 2), g["greater_2_kept"], fails)
    _cmp("golden > -2", compact(a, "greater", -2), g["greater_minus2_kept"], fails)
    # the kept elements sit at the exclusive scan of the selection (Python ints)
    sel = [1 if x != 0 else 0 for x in g["input"]]
    pos = [sum(sel[:i]) for i in range(len(sel))]
    if pos != g["nonzero_positions"] or sel != g["nonzero_selection"]:
        fails.append("fixture positions are not the exclusive scan of the selection")
    rng = np.random.default_rng(90)
    for dt in (np.int32, np.uint32):
        x = rng.integers(np.iinfo(dt).min, np.iinfo(dt).max, size=5000, dtype=np.int64, endpoint=True).astype(dt)
        x[rng.random(x.size) < 0.3] = 0
        thr = dt(rng.integers(np.iinfo(dt).min // 2, np.iinfo(dt).max // 2))
        _cmp("numpy mask nonzero %s" % np.dtype(dt).name, compact(x, "nonzero", 0), x[x != 0], fails)
        _cmp("numpy mask greater %s" % np.dtype(dt).name, compact(x, "greater", thr), x[x > thr], fails)
    f = rng.standard_normal(3000).astype(np.float32)
    f[::97] = np.nan
    got = np.asarray(compact(f, "greater", np.float32(0.25)))
    want = f[f > np.float32(0.25)]
    if got.shape != want.shape or not np.array_equal(got.view(np.uint32), want.view(np.uint32)):
        fails.append("numpy mask float32 greater (NaN never kept)")
    # special cases: nothing kept, everything kept (a copy), empty input
    z = np.zeros(100, dtype=np.int32)
    if np.asarray(compact(z, "nonzero", 0)).size != 0:
        fails.append("all-zero input keeps nothing")
    o = np.arange(1, 101, dtype=np.int32)
    _cmp("everything kept = copy", compact(o, "greater", 0), o, fails)
    if np.asarray(compact(np.zeros(0, dtype=np.int32), "nonzero", 0)).size != 0:
        fails.append("empty input")
    return fails
