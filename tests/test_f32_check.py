"""The float acceptance rule the GPU parity tests use (gpu_util.f32_bad), on
hand-made cases and without a GPU: a NaN or infinite output where the
reference is finite fails, non-finite references are matched by class, and
the comparison of the old form (err > tol, which lets NaN through) is caught
by these cases."""
import numpy as np

from gpu_util import assert_f32_close, f32_bad

NAN, INF = np.nan, np.inf

# (got, ref, abs_sums, should_pass)
CASES = [
    ([1, 2, 3], [1, 2, 3], [1, 2, 3], True),
    ([1, NAN, 3], [1, 2, 3], [1, 2, 3], False),              # NaN output, finite reference
    ([1, INF, 3], [1, 2, 3], [1, 2, 3], False),              # infinite output, finite reference
    ([1, -INF, 3], [1, 2, 3], [1, 2, 3], False),
    ([1, 2 + 2.0**-18, 3], [1, 2, 3], [1, 2, 3], False),     # outside 2^-20 * sum|a| = 2^-19
    ([1, 2 + 2.0**-20, 3], [1, 2, 3], [1, 2, 3], True),      # inside it
    ([1, NAN, NAN], [1, NAN, NAN], [1, NAN, NAN], True),     # NaN where the reference is NaN
    ([1, 2, NAN], [1, NAN, NAN], [1, NAN, NAN], False),      # finite where the reference is NaN
    ([1, INF, INF], [1, INF, INF], [1, INF, INF], True),
    ([1, INF, -INF], [1, INF, INF], [1, INF, INF], False),   # wrong sign of infinity
    ([1, NAN, INF], [1, INF, INF], [1, INF, INF], False),    # NaN where the reference is +inf
    ([-0.0, 0.0], [0.0, -0.0], [0.0, 0.0], True),            # zeros of either sign
]


def _fails(bad_fn):
    out = []
    for k, (got, ref, ab, ok) in enumerate(CASES):
        flagged = bad_fn(np.array(got, dtype=np.float32), np.array(ref, dtype=np.float64),
                         np.array(ab, dtype=np.float64)).size > 0
        if flagged == ok:
            out.append(k)
    return out


def test_acceptance_rule_cases():
    assert _fails(f32_bad) == []


def _old_rule(got, ref, ab):
    # the comparison as first written: a NaN error is never "> tol"
    with np.errstate(invalid="ignore"):
        return np.nonzero(np.abs(got.astype(np.float64) - ref) > np.ldexp(ab, -20))[0]


def test_cases_catch_the_nan_blind_rule():
    assert 1 in _fails(_old_rule)


def test_assert_helper_raises_on_nan():
    try:
        assert_f32_close(np.array([1, NAN, 3], dtype=np.float32), np.array([1.0, 2.0, 3.0]),
                         np.array([1.0, 2.0, 3.0]), "planted NaN")
    except AssertionError as e:
        assert "planted NaN" in str(e)
    else:
        raise AssertionError("a NaN output passed the float acceptance check")
