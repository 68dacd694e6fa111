"""C ABI on the host: the library loads, exports every declared entry point,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi355scan.h")


def _lib():
    from paper_2312_14874_amd import _lib as L
    return L


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scan_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = _lib()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L.lib, name), name
        assert name in L.SIGNATURES, "binding lacks " + name


def test_status_strings():
    L = _lib()
    for code in range(8):
        s = L.lib.scan_status_string(code)
        assert s and s != b"unknown status"
    assert L.lib.scan_status_string(99) == b"unknown status"


INVALID, OVERLAP = 1, 2


@pytest.mark.parametrize("args,code", [
    ((None, None, 10, 0, 0), INVALID),          # null pointers
    ((4096, 8192, -1, 0, 0), INVALID),          # n < 0
    ((4096, 8192, 10, 7, 0), INVALID),          # unknown dtype
    ((4096, 8192, 10, 0, 0x10), INVALID),       # unknown flag
    ((4098, 8192, 10, 0, 0), INVALID),          # misaligned (needs 4 bytes)
    ((4096, 4100, 10, 0, 0), OVERLAP),          # partial overlap
    ((4100, 4096, 10, 2, 1), OVERLAP),
])
def test_flat_argument_errors(args, code):
    L = _lib()
    assert L.lib.scan_flat(*args, None) == code


@pytest.mark.parametrize("args,code", [
    ((None, None, 10, 0, 0), INVALID),          # null pointers
    ((4096, 8192, 10, 0, 0x10), INVALID),       # unknown flag
    ((4096, 4100, 10, 0, 0), OVERLAP),          # partial overlap
    ((4096, 1 << 20, 10, 3, 0), 5),             # 64-bit dtypes: not offered without allocation
    ((4096, 1 << 20, 10, 2, 0x4), 5),           # max of float32
])
def test_noalloc_argument_errors(args, code):
    L = _lib()
    assert L.lib.scan_flat_noalloc(*args, None) == code


# The allocation-free scan holds 32768 tiles: 98,304-element tiles at most for
# 16-byte aligned buffers, 8,192-element tiles otherwise.
NOALLOC_MAX_ALIGNED = 32768 * 98304
NOALLOC_MAX_UNALIGNED = 32768 * 8192


@pytest.mark.parametrize("n,misalign", [(NOALLOC_MAX_ALIGNED + 1, 0), (NOALLOC_MAX_UNALIGNED + 1, 4),
                                        (1 << 40, 0)])
def test_noalloc_rejects_sizes_beyond_its_array(n, misalign):
    # refused on the host before any device call (none is made here: no GPU)
    L = _lib()
    a = (1 << 44) + misalign
    assert L.lib.scan_flat_noalloc(a, a + (1 << 45), n, 1, 0, None) == INVALID
    assert L.lib.scan_flat_noalloc(a, a, n, 2, 1, None) == INVALID


def test_zero_length_is_noop():
    L = _lib()
    assert L.lib.scan_flat(None, None, 0, 0, 0, None) == 0
    assert L.lib.scan_flat_noalloc(None, None, 0, 0, 0, None) == 0
    assert L.lib.scan_inclusive_i32(None, None, 0, None) == 0
    assert L.lib.scan_segmented_batch(None, None, None, 0, 0, 0, 0, None) == 0


def test_segmented_argument_errors():
    L = _lib()
    f = L.lib.scan_segmented_batch
    assert f(4096, 8192, None, 3, 10, 0, 0, None) == INVALID        # no offsets
    assert f(4096, 8192, 16, -1, 10, 0, 0, None) == INVALID         # S < 0
    assert f(4096, 8192, 16, 0, 10, 0, 0, None) == INVALID          # S = 0 with n > 0
    assert f(4096, 8192, 20, 3, 10, 0, 0, None) == INVALID          # offsets misaligned
    assert f(4096, 4100, 16, 3, 10, 0, 0, None) == OVERLAP


NOT_SUPPORTED = 5
OP_MAX, OP_MIN, OP_XOR, REV, EXC = 0x4, 0x8, 0xC, 0x2, 0x1


@pytest.mark.parametrize("dtype,flags", [
    (2, OP_MAX), (2, OP_MIN), (2, OP_XOR),       # float32 takes + only
    (0, OP_MIN | REV), (1, OP_MIN | REV),        # reverse with a nonzero identity
    (0, OP_MAX | REV),
])
def test_operator_not_supported(dtype, flags):
    L = _lib()
    assert L.lib.scan_flat(4096, 8192, 10, dtype, flags, None) == NOT_SUPPORTED
    assert L.lib.scan_segmented_batch(4096, 8192, 16, 1, 10, dtype, flags, None) == NOT_SUPPORTED


def test_operator_argument_errors_first():
    L = _lib()
    # bad arguments are reported before an unsupported operator combination
    assert L.lib.scan_flat(None, None, 10, 2, OP_MAX, None) == INVALID
    assert L.lib.scan_flat(None, None, 0, 0, OP_MAX | EXC, None) == 0
    assert L.lib.scan_two_pass(4096, 8192, 10, 0, OP_XOR, 1, 0, None) == NOT_SUPPORTED


def test_compact_argument_errors():
    L = _lib()
    f = L.lib.scan_compact
    assert f(4096, 8192, 10, 0, 0, 0, None, None) == INVALID        # no count pointer
    assert f(4096, 8192, 10, 0, 0, 0, 12, None) == INVALID          # count misaligned
    assert f(4096, 8192, 10, 0, 2, 0, 16, None) == INVALID          # unknown predicate
    assert f(None, None, 10, 0, 0, 0, 16, None) == INVALID          # null pointers
    assert f(4096, 4100, 10, 0, 0, 0, 16, None) == OVERLAP
    assert f(4096, 8192, 10, 7, 0, 0, 16, None) == INVALID          # unknown dtype
    assert f(1 << 40, 1 << 41, 1 << 33, 0, 0, 0, 16, None) == NOT_SUPPORTED   # n >= 2^32


def test_partition_argument_errors():
    L = _lib()
    f = L.lib.scan_partition
    assert f(4096, 8192, 10, 0, 0, 0, None, None) == INVALID        # no count pointer
    assert f(4096, 8192, 10, 0, 2, 0, 16, None) == INVALID          # unknown predicate
    assert f(4096, 4096, 10, 0, 0, 0, 16, None) == OVERLAP          # in place is refused
    assert f(4096, 4100, 10, 0, 0, 0, 16, None) == OVERLAP
    assert f(4096, 8192, 10, 3, 0, 0, 16, None) == NOT_SUPPORTED    # 64-bit dtypes
    assert f(1 << 40, 1 << 41, 1 << 33, 0, 0, 0, 16, None) == NOT_SUPPORTED   # n >= 2^32


def test_two_pass_argument_errors():
    L = _lib()
    f = L.lib.scan_two_pass
    assert f(None, None, 0, 0, 0, 0, 0, None) == 0                  # n = 0: no-op
    assert f(None, None, 10, 0, 0, 0, 0, None) == INVALID           # null pointers
    assert f(4096, 8192, 10, 0, 0, 2, 0, None) == INVALID           # unknown method
    assert f(4096, 8192, 10, 0, 0, 1, -1, None) == INVALID          # partition < 0
    assert f(4096, 8192, 10, 7, 0, 1, 0, None) == INVALID           # unknown dtype
    assert f(4096, 4100, 10, 0, 0, 1, 0, None) == OVERLAP
    assert f(4096, 8192, 10, 0, 2, 1, 0, None) == 5                 # reverse: not supported


I64, U64, F64 = 3, 4, 5


def test_int64_argument_errors():
    L = _lib()
    f = L.lib.scan_flat
    assert f(None, None, 0, I64, 0, None) == 0                      # n = 0: no-op
    assert f(None, None, 10, I64, 0, None) == INVALID               # null pointers
    assert f(4100, 8192, 10, U64, 0, None) == INVALID               # not 8-byte aligned
    assert f(4104, 8192, 10, I64, 0, None) == INVALID               # 8- but not 16-byte aligned
    assert f(4096, 4136, 10, I64, 0, None) == OVERLAP               # 8-byte elements overlap
    assert f(4096, 8192, 10, U64, OP_MAX, None) == NOT_SUPPORTED    # + only
    assert f(4096, 8192, 10, I64, 0x10, None) == INVALID            # unknown flag
    assert f(4104, 8192, 10, F64, 0, None) == INVALID               # float64: 16-byte alignment too
    assert f(4096, 8192, 10, F64, OP_XOR, None) == NOT_SUPPORTED
    # the other entry points take 32-bit dtypes only
    assert L.lib.scan_segmented_batch(4096, 8192, 16, 1, 10, I64, 0, None) == NOT_SUPPORTED
    assert L.lib.scan_two_pass(4096, 8192, 10, U64, 0, 1, 0, None) == NOT_SUPPORTED
    assert L.lib.scan_compact(4096, 8192, 10, I64, 0, 0, 16, None) == NOT_SUPPORTED
    assert L.lib.scan_segmented_batch(4096, 8192, 16, 1, 10, F64, 0, None) == NOT_SUPPORTED
    assert L.lib.scan_selected_config(F64, 0, 0, 100) == -1


def test_other_argument_errors():
    L = _lib()
    assert L.lib.scan_reserve(-1, None) == INVALID
    assert L.lib.scan_reserve(0, None) == 0
    assert L.lib.scan_graph_launch(None, None) == INVALID
    assert L.lib.scan_graph_destroy(None) == INVALID
    assert L.lib.scan_force_config(10_000) == INVALID
    assert L.lib.scan_config_info(-1, None, None, None, None, None, None) == INVALID
    assert L.lib.scan_segmented_looped(4096, 8192, None, 2, 0, 0, None) == INVALID
    h = ctypes.c_void_p()
    assert L.lib.scan_looped_graph_create(4096, 8192, None, 2, 0, 0, None, ctypes.byref(h)) == INVALID


def test_configs_are_well_formed():
    from paper_2312_14874_amd import config_info, num_configs
    n = num_configs()
    assert n >= 10
    for c in range(n):
        info = config_info(c)
        assert info["block"] % 64 == 0 and info["items"] % 4 == 0
        assert 2048 <= info["tile"] <= 131072 and info["mode"] in (0, 1, 2, 4)
        assert info["per_cu"] >= 0 and 1 <= info["cu_pct"] <= 100


def test_tune_file_roundtrip(tmp_path):
    from paper_2312_14874_amd import config_info, force_config, lib, selected_config, tune_load, tune_save
    import torch
    p = tmp_path / "t.json"
    info = config_info(5)
    p.write_text('{"arch": "gfx950", "entries": [{"op": "int", "segmented": 0, "log2n": 20, '
                 '"config": 5, "block": %d, "items": %d}, '
                 '{"op": "f32", "segmented": 1, "log2n": 21, "config": 5, "block": 1, "items": 1}]}'
                 % (info["block"], info["items"]))
    tune_load(str(p))
    assert selected_config(torch.int32, 1 << 20) == 5
    assert selected_config(torch.int32, (1 << 21) - 1) == 5
    # mismatching block/items are ignored
    assert selected_config(torch.float32, 1 << 21, segmented=True) != 5
    tune_save(str(tmp_path / "u.json"))
    assert '"config": 5' in (tmp_path / "u.json").read_text()
    force_config(3)
    assert selected_config(torch.int32, 1 << 20) == 3
    force_config(-1)
    # restore the shipped table
    from paper_2312_14874_amd import _lib as L
    shipped = os.path.join(os.path.dirname(L.LIB_PATH), "tune", "gfx950.json")
    if os.path.exists(shipped):
        tune_load(shipped)
    else:
        p.write_text('{"entries": []}')
        tune_load(str(p))
    assert lib.scan_tune_load(str(tmp_path / "missing.json").encode()) == INVALID


@pytest.mark.parametrize("args,code", [
    ((4096, 1 << 20, 10, -1), INVALID),       # unknown configuration
    ((4096, 1 << 20, 10, 10 ** 6), INVALID),
    ((4100, 1 << 20, 10, 22), INVALID),       # not 16-byte aligned
    ((4096, 4100, 10, 22), OVERLAP),          # partial overlap
    ((4096, 1 << 20, 10, 0), 5),              # tile = workgroup index: not a counter mode
    ((4096, 1 << 20, 10, 8), 5),              # static round robin: not a counter mode
    ((None, None, 0, 22), 0),                 # n = 0
])
def test_stream_ceiling_argument_errors(args, code):
    L = _lib()
    assert L.lib.scan_stream_ceiling(*args, None) == code
