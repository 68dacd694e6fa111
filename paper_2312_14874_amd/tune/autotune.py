"""Autotuner: time every kernel configuration per (dtype, segmented, log2 n)
bucket on this GPU and write the tuning table the library loads at start-up.

    python -m paper_2312_14874_amd.tune.autotune [--out FILE] [--min 10] [--max 30]

The tile (threads x items per thread) is the GPU counterpart of the paper's
cache-sized partition (Section 2.2), whose best size the paper finds by a sweep
(Section 4.2.4); here the sweep also covers workgroup size, non-temporal hints
and a persistent grid.  Timing uses HIP events on the stream of the calls,
median of `reps` runs after one warm-up, with rotating buffers for sizes the
256 MB Infinity Cache could hold.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

import numpy as np
import torch

from .. import _lib
from ..ops import config_info, force_config, num_configs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "gfx950.json")


def _loguniform_offsets(rng, n, lo=1, hi=1 << 20):
    """Segment offsets covering n elements with log-uniform lengths in [lo, hi]."""
    lens = []
    total = 0
    while total < n:
        L = int(np.clip(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1)))), lo, hi))
        L = min(L, n - total)
        lens.append(L)
        total += L
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def time_config(cfg, bufs, dtype_code, flags, seg_offsets, reps, stream):
    """Median kernel time (ms) of configuration cfg over rotating buffers, each
    launch between its own pair of HIP events; the GPU is kept busy while the
    host enqueues, so that no launch waits for the host between its events."""
    L = _lib.lib
    force_config(cfg)

    def launch(i):
        x, y = bufs[i % len(bufs)]
        if seg_offsets is None:
            s = L.scan_flat(x.data_ptr(), y.data_ptr(), x.numel(), dtype_code, flags, stream)
        else:
            s = L.scan_segmented_batch(x.data_ptr(), y.data_ptr(), seg_offsets.data_ptr(),
                                       seg_offsets.numel() - 1, x.numel(), dtype_code, flags, stream)
        _lib.check(s, "tuning launch")

    try:
        launch(0)                                   # warm-up (and workspace growth)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        torch.cuda._sleep(int(max(reps * 60e-6, 2e-3) * 2.4e9))
        for i in range(reps):
            ev[i][0].record()
            launch(i + 1)
            ev[i][1].record()
        torch.cuda.synchronize()
        ts = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        return ts[len(ts) // 2]
    finally:
        force_config(-1)


def sweep(n, dtype="int", segmented=False, reps=11, verbose=True, seed=0):
    dev = torch.device("cuda", torch.cuda.current_device())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    tdt = torch.float32 if dtype == "f32" else torch.int32
    code = _lib.SCAN_F32 if dtype == "f32" else _lib.SCAN_I32
    nbuf = max(1, min(8, (1 << 29) // max(1, 8 * n)))   # > 512 MiB in rotation for small n
    bufs = []
    for _ in range(nbuf):
        x = torch.randn(n, device=dev) if dtype == "f32" else torch.randint(0, 100, (n,), device=dev, dtype=tdt)
        bufs.append((x, torch.empty_like(x)))
    offs = None
    flags = 0
    if segmented:
        offs = torch.from_numpy(_loguniform_offsets(np.random.default_rng(seed), n)).to(dev)
        flags = _lib.SCAN_EXCLUSIVE
    res = []
    for cfg in range(num_configs()):
        ms = time_config(cfg, bufs, code, flags, offs, reps, stream)
        res.append((ms, cfg))
        if verbose:
            info = config_info(cfg)
            print("  n=2^%-2d %-3s seg=%d cfg %2d (block %4d items %2d nt %d mode %d): %9.2f us  %7.1f GB/s"
                  % (int(np.log2(n)), dtype, segmented, cfg, info["block"], info["items"], info["nontemporal"],
                     info["mode"], ms * 1e3, 8 * n / (ms * 1e-3) / 1e9), file=sys.stderr, flush=True)
    return pick(res), res


# A configuration whose tile order relies on the dispatcher (mode 2: tile =
# workgroup index, in-order dispatch assumed) or on co-residency (mode 4) is
# taken only when it beats the best counter-mode configuration by more than
# this fraction (the library's scan_autotune applies the same rule).
ORDERED_MARGIN = 0.03


def pick(res):
    """The fastest configuration of res [(ms, cfg)], preferring counter modes
    (0, 1) unless another mode wins by more than ORDERED_MARGIN."""
    best_ms, best = min(res)
    dyn = [(ms, c) for ms, c in res if config_info(c)["mode"] in (0, 1)]
    if not dyn:
        return best
    dyn_ms, dyn_best = min(dyn)
    return best if best_ms < dyn_ms * (1.0 - ORDERED_MARGIN) else dyn_best


def merge_keep(entries, dtypes, segmented, lo, hi):
    """The entries of an existing table that a run tuning the given dtypes,
    segmented flags and log2 n buckets lo..hi leaves in place."""
    return [e for e in entries
            if not (e["op"] in dtypes and e["segmented"] in segmented and lo <= e["log2n"] <= hi)]


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--out", default=DEFAULT_OUT)
    p.add_argument("--min", type=int, default=10)
    p.add_argument("--max", type=int, default=30)
    p.add_argument("--reps", type=int, default=11)
    p.add_argument("--dtypes", default="int,f32")
    p.add_argument("--segmented", default="0,1")
    p.add_argument("--merge", action="store_true",
                   help="keep the entries of --out for the buckets not tuned now")
    args = p.parse_args()
    entries = []
    if args.merge and os.path.exists(args.out):
        with open(args.out) as f:
            entries = merge_keep(json.load(f)["entries"], args.dtypes.split(","),
                                 [int(s) for s in args.segmented.split(",")], args.min, args.max)
    for dtype in args.dtypes.split(","):
        for seg in [int(s) for s in args.segmented.split(",")]:
            for b in range(args.min, args.max + 1):
                best, _ = sweep(1 << b, dtype, bool(seg), args.reps)
                info = config_info(best)
                entries.append({"op": dtype, "segmented": seg, "log2n": b, "config": best,
                                "block": info["block"], "items": info["items"],
                                "nontemporal": info["nontemporal"], "mode": info["mode"]})
                print("best n=2^%d %s seg=%d: config %d" % (b, dtype, seg, best), file=sys.stderr, flush=True)
    entries.sort(key=lambda e: (e["op"] != "int", e["segmented"], e["log2n"]))
    with open(args.out, "w") as f:
        json.dump({"arch": "gfx950", "format": 1, "entries": entries}, f, indent=1)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
