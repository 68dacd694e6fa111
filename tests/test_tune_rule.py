"""The autotuners' rule for tile modes that rely on the dispatcher (mode 2,
tile = workgroup index) or on co-residency (mode 4): such a configuration is
chosen only when it beats the best counter-mode configuration by more than 3%
(no GPU needed: the rule is applied to given timings)."""
import pytest


def _modes():
    from paper_2312_14874_amd import config_info, num_configs
    by_mode = {}
    for c in range(num_configs()):
        by_mode.setdefault(config_info(c)["mode"], []).append(c)
    return by_mode


def test_ordered_config_needs_a_clear_win():
    from paper_2312_14874_amd.tune.autotune import ORDERED_MARGIN, pick
    m = _modes()
    ordered, static, counter, resident = m[2][0], m[4][0], m[0][0], m[1][0]
    assert ORDERED_MARGIN == pytest.approx(0.03)
    # within the margin: the fastest counter-mode configuration wins
    assert pick([(0.990, ordered), (1.000, resident), (1.010, counter)]) == resident
    assert pick([(0.975, static), (1.000, counter), (1.100, resident)]) == counter
    # a clear win: the ordered / static configuration is taken
    assert pick([(0.950, ordered), (1.000, resident)]) == ordered
    assert pick([(0.900, static), (1.000, counter)]) == static
    # counter modes compete on time alone
    assert pick([(1.000, resident), (0.999, counter)]) == counter


def test_merge_replaces_only_the_buckets_tuned():
    from paper_2312_14874_amd.tune.autotune import merge_keep
    table = [{"op": op, "segmented": sg, "log2n": b, "config": 0}
             for op in ("int", "f32") for sg in (0, 1) for b in range(10, 31)]
    kept = merge_keep(table, ["f32"], [0], 26, 30)
    gone = [e for e in table if e not in kept]
    assert len(gone) == 5
    assert all(e["op"] == "f32" and e["segmented"] == 0 and 26 <= e["log2n"] <= 30 for e in gone)
    # every bucket of a family tuned in full
    assert len(merge_keep(table, ["int", "f32"], [1], 10, 30)) == 2 * 21
