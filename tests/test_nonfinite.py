"""Non-finite float inputs on the GPU against the oracle.

Reading of the definition for IEEE inputs: an output is NaN when its prefix
(suffix for reverse scans; its own segment only for segmented scans) holds a
NaN or both infinities, +inf / -inf when it holds only that infinity, and
otherwise the finite sum within the usual bound; zeros of either sign compare
equal.  Inputs are normal(0, 1) with NaN / infinities planted at seeded
positions, so the non-finite values travel through lanes, chunk and wave
totals, tile status words and the carries of later tiles."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_f32_close, configs, f32_bad, flat, segmented

pytestmark = pytest.mark.gpu

try:
    from paper_2312_14874_amd import num_configs
    NUM_CONFIGS = num_configs()
except ImportError:   # library not built: the GPU tests cannot run anyway
    NUM_CONFIGS = 1

NAN, INF = np.nan, np.inf
PATTERNS = {
    "nan": [NAN],
    "pos_inf": [INF],
    "neg_inf": [-INF],
    "both_inf": [INF, -INF],
    "inf_then_nan": [INF, NAN],
}


def planted(n, seed, kinds, dtype=np.float32):
    g = np.random.default_rng(seed)
    a = g.standard_normal(n).astype(dtype)
    a[g.integers(0, n, size=len(kinds))] = np.array(kinds, dtype=dtype)
    return a


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_flat_nonfinite_every_config(cfg):
    tile = configs()[cfg]["tile"]
    n = 5 * tile + 77
    for k, (name, kinds) in enumerate(PATTERNS.items()):
        a = planted(n, 300 + 10 * cfg + k, kinds)
        for ex in (False, True):
            for rev in (False, True):
                got = flat(a, exclusive=ex, reverse=rev, cfg=cfg)
                ref, ab = oracle.scan_f32(a, exclusive=ex, reverse=rev)
                assert_f32_close(got, ref, ab, "cfg %d %s ex %d rev %d" % (cfg, name, ex, rev))


def test_flat_nonfinite_default_config_large():
    # the configuration the library selects, many tiles after the planted values
    n = (1 << 24) + 3
    for k, (name, kinds) in enumerate(PATTERNS.items()):
        a = planted(n, 400 + k, kinds)
        for ex in (False, True):
            for rev in (False, True):
                got = flat(a, exclusive=ex, reverse=rev)
                ref, ab = oracle.scan_f32(a, exclusive=ex, reverse=rev)
                assert_f32_close(got, ref, ab, "%s ex %d rev %d" % (name, ex, rev))


def test_negative_zeros():
    for n in (1, 300, 3 * 98304 + 5):
        a = np.full(n, -0.0, dtype=np.float32)
        for ex in (False, True):
            for rev in (False, True):
                got = flat(a, exclusive=ex, reverse=rev)
                assert np.all(got == 0.0), "n %d ex %d rev %d" % (n, ex, rev)


@pytest.mark.parametrize("cfg", range(NUM_CONFIGS))
def test_segmented_nonfinite_every_config(cfg):
    tile = configs()[cfg]["tile"]
    n = 7 * tile + 11
    g = np.random.default_rng(500 + cfg)
    off = workloads.random_offsets(g, n, 40)
    for k, (name, kinds) in enumerate(PATTERNS.items()):
        a = planted(n, 600 + 10 * cfg + k, kinds * 3)
        for ex in (False, True):
            for rev in (False, True):
                got = segmented(a, off, exclusive=ex, reverse=rev, cfg=cfg)
                ref, ab = oracle.segmented_f32(a, off, exclusive=ex, reverse=rev)
                assert_f32_close(got, ref, ab, "cfg %d %s ex %d rev %d" % (cfg, name, ex, rev))


def test_two_pass_nonfinite():
    torch = pytest.importorskip("torch")
    import paper_2312_14874_amd as scan
    n = 3_000_017
    for k, (name, kinds) in enumerate(PATTERNS.items()):
        a = planted(n, 700 + k, kinds)
        x = torch.from_numpy(a).cuda()
        for method in ("prefix_increment", "accumulate_prefix"):
            for part in (0, 1 << 20):
                for ex in (False, True):
                    got = scan.two_pass_cumsum(x, method, exclusive=ex, partition=part).cpu().numpy()
                    ref, ab = oracle.scan_f32(a, exclusive=ex)
                    assert_f32_close(got, ref, ab, "%s %s part %d ex %d" % (name, method, part, ex))


def test_f64_nonfinite():
    torch = pytest.importorskip("torch")
    import paper_2312_14874_amd as scan
    n = 5 * 32768 + 19
    depth = 8 * (-(-n // 32768)) + 128
    for k, (name, kinds) in enumerate(PATTERNS.items()):
        a = planted(n, 800 + k, kinds, dtype=np.float64)
        x = torch.from_numpy(a).cuda()
        for ex in (False, True):
            for rev in (False, True):
                got = scan.cumsum(x, exclusive=ex, reverse=rev).cpu().numpy()
                ref, ab = oracle.scan_f64(a, exclusive=ex, reverse=rev)
                bad = f32_bad(got, ref, ab * (depth + 1) * (1 + 1e-6), exp=-53)
                assert bad.size == 0, "%s ex %d rev %d: %d bad, first %d: got %r ref %r" % (
                    name, ex, rev, bad.size, bad[0], got[bad[0]], ref[bad[0]])
