"""Benchmark: single-pass int32/uint32 inclusive scan at n = 2^28 on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

A step is one inclusive scan of n = 2^28 full-range uint32 values (wrapping
modulo 2^32; int32 is the same kernel on the same bits), out of place, inputs
resident in HBM.  Prints ONE JSON line on stdout; progress goes to stderr.

  value      whole-job throughput in GB/s of algorithmic traffic (8 bytes per
             element: one 4-byte read and one 4-byte write), from the wall
             clock of the K timed steps
  roofline   the scan kernel's average duration from HIP events on the stream
             it runs on, against the 8 TB/s HBM peak; `traffic` is the HBM
             bytes per launch measured with rocprofv3 counters (profiles/),
             or null when the kernel sources changed since that measurement
  cpu_baseline  the sequential oracle on one host core, over repeated passes
             of the same 2^28-element input (about 10 s); its output also
             checks the timed GPU result.  The CPU legs run last and are the
             only part of this script that calls the oracle.
  cpu_context the paper's own multithreaded scheme (Accumulate + Prefix Sum
             over cache-sized partitions, one barrier per iteration) on up to
             16 host cores, same input, checked against the oracle; context
             beside cpu_baseline, not a target
  segmented  the batched segmented scan (4096 segments, log-uniform lengths in
             [1, 2^20], Poisson(8) int32 counts, exclusive, one persistent
             launch replayed from a hipGraph) against one flat-scan launch per
             segment, eager and graph-captured; the batched result is checked
             exactly on the GPU (0 at each segment start, y[i] = y[i-1] +
             x[i-1] elsewhere) and the others must equal it
  two_pass   the same n = 2^28 scan by the paper's two-pass algorithms
             (Section 2.1: Prefix Sum + Increment, Accumulate + Prefix Sum),
             whole-array and over cache-sized partitions (Section 2.2),
             against the single pass; results compared with its output
  operators  the same input scanned with max, min and xor (int32), kernel
             time from HIP events, each result checked exactly on the GPU by
             its recurrence y[i] = y[i-1] op x[i]
  compaction the same input read as int32, elements > 0 kept (about half)
             by the fused one-pass compaction, against torch's masked select
             for context; the result must equal torch's.  Also the two-way
             partition of the same input (kept first, the rest reversed after
             them), whose halves must equal torch's masked selects
  wide       64-bit elements, n = 2^28: uint64 full-range values (the bench
             input as high halves, reversed as low halves) and float64
             normal(0,1), inclusive, kernel time from HIP events at 16 bytes
             per element; uint64 checked exactly by its recurrence on the GPU,
             float64 against the oracle within its bound in the CPU legs
  ceiling    the streaming-ceiling kernel (out = in + 1 with the scan's tiles,
             accesses, resident grid and store/load hand-off, but no scan and
             no look-back) over every counter-mode configuration on the same
             input; frac_copy = the scan's GB/s over the best of them, and over
             the one of the scan's own configuration; each result checked
             exactly (y = x + 1) on the GPU
  sizes      the other sizes of the workloads: 2^20 int32 in [0, 100)
             inclusive and exclusive (64 rotating buffer pairs), the uint32
             bandwidth curve at 2^24 (8 rotating pairs), 2^28 in place and 2^30;
             kernel time per launch from HIP events (median, p10, p90), each
             result checked exactly on the GPU by its recurrence
  float32    inclusive scan of 2^28 float32 normal(0,1) (seed 1003), checked
             against the oracle within 2^-20 * sum|a| in the CPU legs
  autograd   the differentiable cumsum on 64 ragged rows (lengths log-uniform
             in [2^10, 2^22], seed 1005): forward (segmented inclusive scan) and
             backward (segmented reverse scan) kernel times, and one
             forward + backward through torch.autograd; both results checked
             against the oracle in the CPU legs
Extra modes (not the headline line): --n, --dtype f32, --copy-calibration.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "scan_u32_n2p28_traffic.txt")
KERNEL_SOURCES = ["paper_2312_14874_amd/csrc/scan_device.hpp", "paper_2312_14874_amd/csrc/scan_shared.hpp",
                  "paper_2312_14874_amd/csrc/scan_kernels.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(n: int):
    """HBM bytes per launch from the committed counter summary, or None if it
    does not match the current kernel sources or this n."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha") != kernel_source_sha() or int(kv.get("n", -1)) != n:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=1 << 28)
    p.add_argument("--dtype", choices=["u32", "f32"], default="u32")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    p.add_argument("--no-segmented", action="store_true", help="skip the segmented comparison")
    p.add_argument("--no-two-pass", action="store_true", help="skip the two-pass comparison")
    p.add_argument("--no-operators", action="store_true", help="skip the max / min / xor scans")
    p.add_argument("--no-compaction", action="store_true", help="skip the stream compaction")
    p.add_argument("--no-wide", action="store_true", help="skip the 64-bit scans")
    p.add_argument("--no-ceiling", action="store_true", help="skip the streaming-ceiling sweep")
    p.add_argument("--no-sizes", action="store_true", help="skip the other sizes (2^20, 2^24, in place, 2^30)")
    p.add_argument("--no-float32", action="store_true", help="skip the float32 scan at 2^28")
    p.add_argument("--no-autograd", action="store_true", help="skip the autograd rows")
    p.add_argument("--no-graphs", action="store_true",
                   help="segmented leg: eager launches only (no graph replays; rocprofv3's counter mode "
                        "does not survive graph launches)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="run only plain device copies of the scan's bytes (counter calibration)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    import paper_2312_14874_amd as scan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    n = args.n
    props = torch.cuda.get_device_properties(dev)
    log("device:", props.name, getattr(props, "gcnArchName", ""), "CUs", props.multi_processor_count)

    if args.copy_calibration:
        # plain copies of exactly the scan's per-launch bytes: n*4 read, n*4 written
        x = torch.empty(n, dtype=torch.int32, device=dev).random_()
        y = torch.empty_like(x)
        for _ in range(args.warmup + args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        log("copy: %d bytes read + %d written per launch, %.1f us, %.1f GB/s"
            % (4 * n, 4 * n, ms * 1e3, 8 * n / (ms * 1e-3) / 1e9))
        return

    # ---------------------------------------------------------- input, resident in HBM
    t0 = time.time()
    if args.dtype == "u32":
        a = workloads.full_u32(n)
        x = torch.from_numpy(a.view(np.int32)).to(dev)
        dtype_code, dtype_name = scan.SCAN_U32, "u32"
    else:
        a = workloads.normal_f32(n)
        x = torch.from_numpy(a).to(dev)
        dtype_code, dtype_name = scan.SCAN_F32, "f32"
    y = torch.empty_like(x)
    log("input ready (%.1f s)" % (time.time() - t0))
    stream = torch.cuda.current_stream(dev)
    sptr = __import__("ctypes").c_void_p(stream.cuda_stream)

    def step():
        s = scan.lib.scan_flat(x.data_ptr(), y.data_ptr(), n, dtype_code, 0, sptr)
        if s != 0:
            raise scan.ScanError(s, "scan_flat")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---------------------------------------------------------- timed region
    K = args.steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(K):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    kern_ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    kern_avg_ms = sum(kern_ms) / K
    ms_per_step = wall * 1e3 / K
    alg_bytes = 8.0 * n
    value = alg_bytes / (ms_per_step * 1e-3) / 1e9
    achieved = alg_bytes / (kern_avg_ms * 1e-3) / 1e9
    log("scan: %.1f us/step wall, kernel avg %.1f us (p10 %.1f, p90 %.1f), %.1f GB/s"
        % (ms_per_step * 1e3, kern_avg_ms * 1e3, kern_ms[K // 10] * 1e3, kern_ms[(9 * K) // 10] * 1e3, achieved))

    # ---------------------------------------------------------- parity of the timed output
    # an inclusive integer +-scan is characterised exactly by y[0] = x[0] and
    # y[i] - y[i-1] = x[i] (mod 2^32): checked on the GPU, no reference needed;
    # the float32 mode is compared with the oracle in the CPU leg
    got = y.cpu().numpy()
    if args.dtype == "u32":
        parity = "bit-exact (y[0]=x[0], y[i]-y[i-1]=x[i])" if inclusive_sum_holds(torch, x, y) else "MISMATCH"
    else:
        parity = "unchecked (--no-cpu)"
    log("parity:", parity)

    # ---------------------------------------------------------- streaming ceiling of the access pattern
    ceil = None
    scan_cfg = scan.selected_config(torch.int32 if args.dtype == "u32" else torch.float32, n)
    if not args.no_ceiling and args.dtype == "u32":
        ceil = ceiling_runs(scan, torch, x, y, stream, scan_cfg, achieved)

    # ---------------------------------------------------------- segmented vs per-launch
    seg = None
    if not args.no_segmented and args.dtype == "u32":
        seg = segmented_comparison(scan, torch, np, workloads, dev, graphs=not args.no_graphs)

    # ---------------------------------------------------------- two-pass algorithms vs the single pass
    two = None
    if not args.no_two_pass and args.dtype == "u32":
        two = two_pass_comparison(scan, torch, x, y, kern_ms[K // 2], stream)

    # ---------------------------------------------------------- other operators on the same input
    ops = None
    if not args.no_operators and args.dtype == "u32":
        ops = operator_runs(scan, torch, x, y, stream)

    # ---------------------------------------------------------- stream compaction of the same input
    comp = None
    if not args.no_compaction and args.dtype == "u32":
        comp = compaction_run(scan, torch, x, y, stream)

    # ---------------------------------------------------------- the other sizes (in place at n)
    sizes = None
    if not args.no_sizes and args.dtype == "u32":
        sizes = size_runs(scan, torch, np, workloads, x, y, stream)

    del x, y
    # ---------------------------------------------------------- float32 and autograd (checked in the CPU legs)
    f32, f32_data, ag, ag_data = None, None, None, None
    if not args.no_float32 and args.dtype == "u32":
        f32, f32_data = float32_run(scan, torch, workloads, stream)
    if not args.no_autograd and args.dtype == "u32":
        ag, ag_data = autograd_run(scan, torch, workloads, stream)

    # ---------------------------------------------------------- 64-bit elements
    wide, wide_f64 = None, None
    if not args.no_wide and args.dtype == "u32":
        wide, wide_f64 = wide_runs(scan, torch, np, a, stream)

    # ---------------------------------------------------------- CPU legs (the oracle on the host)
    cpu, cpu_ctx = None, None
    if not args.no_cpu:
        cpu, cpu_ctx, f64_ok = cpu_legs(args, np, a, got, alg_bytes, wide_f64)
        cpu.update(host_info())
        if args.dtype == "f32":
            parity = "within 2^-20*sum|a|" if cpu["gpu_result_within_bound"] else "MISMATCH"
        if wide is not None:
            wide["f64_vs_oracle"] = f64_ok
        if f32 is not None:
            f32["within_bound_vs_oracle"] = float32_check(np, *f32_data)
        if ag is not None:
            ag.update(autograd_check(np, *ag_data))
    del wide_f64, f32_data, ag_data

    traffic = measured_traffic(n) if args.dtype == "u32" else None
    out = {
        "metric": "int32 scan GB/s at n=2^28 vs HBM peak; batched-segmented vs per-launch",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic",
        "config": {"workload": "inclusive scan, n=2^%d %s (%s), out of place, single pass"
                               % (n.bit_length() - 1, "uint32 full-range, wrapping" if args.dtype == "u32"
                                  else "float32 normal(0,1)", "seed %d" % (1002 if args.dtype == "u32" else 1003)),
                   "n": n, "scan_config": scan_cfg,
                   "parity": parity},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_GBS, 4), "traffic": traffic,
                     "kernel_avg_us": round(kern_avg_ms * 1e3, 2), "algorithmic_bytes": int(alg_bytes),
                     "Gelem_per_s": round(n / (kern_avg_ms * 1e-3) / 1e9, 2),
                     "frac_copy": ceil["frac_copy"] if ceil else None,
                     "frac_copy_same_config": ceil["frac_copy_same_config"] if ceil else None},
        "cpu_baseline": cpu,
        "cpu_context": cpu_ctx,
        "ceiling": ceil,
        "sizes": sizes,
        "float32": f32,
        "autograd": ag,
        "segmented": seg,
        "two_pass": two,
        "operators": ops,
        "compaction": comp,
        "wide": wide,
    }
    print(json.dumps(out), flush=True)


def host_info():
    """The host the CPU legs ran on: CPU model and core counts."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"host_cpu": model, "host_nproc": os.cpu_count(), "host_cpus_usable": len(os.sched_getaffinity(0))}


def ceiling_runs(scan, torch, x, y, stream, scan_cfg, scan_GBps):
    """The streaming-ceiling kernel (the scan's memory access pattern without
    the scan) on the bench input, over every counter-mode configuration; each
    result is checked exactly (y = x + 1 modulo 2^32)."""
    import ctypes
    n = x.numel()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    runs, exact = [], True
    for c in range(scan.num_configs()):
        info = scan.config_info(c)
        if info["mode"] not in (0, 1):
            continue

        def run():
            scan.check(scan.lib.scan_stream_ceiling(x.data_ptr(), y.data_ptr(), n, c, sptr), "scan_stream_ceiling")
        run()
        torch.cuda.synchronize()
        exact = exact and bool(torch.equal(y, x + 1))
        ms = _median_ms(torch, run, stream, 10)
        runs.append({"config": c, "block": info["block"], "items": info["items"], "per_cu": info["per_cu"],
                     "cu_pct": info["cu_pct"], "us": round(ms * 1e3, 1),
                     "GBps": round(8.0 * n / (ms * 1e-3) / 1e9, 1)})
    best = max(runs, key=lambda r: r["GBps"])
    same = next((r for r in runs if r["config"] == scan_cfg), None)
    res = {"workload": "out = in + 1 over the same n=2^%d input with the scan's tiles, accesses, grid and "
                       "store/load hand-off, no scan and no look-back" % (n.bit_length() - 1),
           "best_config": best["config"], "best_us": best["us"], "best_GBps": best["GBps"],
           "frac_copy": round(scan_GBps / best["GBps"], 4),
           "same_config": scan_cfg, "same_config_us": same["us"] if same else None,
           "same_config_GBps": same["GBps"] if same else None,
           "frac_copy_same_config": round(scan_GBps / same["GBps"], 4) if same else None,
           "runs": runs, "results_exact": exact}
    log("ceiling: best config %d %.1f GB/s, scan's config %s %s GB/s" % (
        best["config"], best["GBps"], scan_cfg, same["GBps"] if same else None))
    return res


def _per_launch_ms(torch, fns, stream, reps):
    """Kernel time of each launch from its own pair of HIP events on the
    stream; launch i runs fns[i % len(fns)] (rotating buffers)."""
    for f in fns:
        f()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    # keep the GPU busy while the host enqueues, so that no launch waits for
    # the host between its two events (a few tens of microseconds per call)
    torch.cuda._sleep(int(max(reps * 60e-6, 5e-3) * 2.4e9))
    for i in range(reps):
        ev[i][0].record(stream)
        fns[i % len(fns)]()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    ts = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return ts[len(ts) // 2], ts[reps // 10], ts[(9 * reps) // 10]


def size_runs(scan, torch, np, workloads, x, y, stream):
    """2^20 int32 in [0, 100) inclusive and exclusive; uint32 full-range at
    2^24, 2^28 in place (on the bench input) and 2^30.  Inputs below 2^25
    elements rotate over enough buffer pairs (>= 512 MiB) that the 256 MB
    last-level cache cannot serve repeated launches.  Each result is checked
    exactly on the GPU: inclusive y[0] = x[0], y[i] - y[i-1] = x[i];
    exclusive y[0] = 0, y[i] - y[i-1] = x[i-1] (modulo 2^32)."""
    dev = x.device
    rows = []

    def row(name, n, t, exact, nbuf):
        ms, p10, p90 = t
        r = {"case": name, "n": n, "us": round(ms * 1e3, 2), "p10_us": round(p10 * 1e3, 2),
             "p90_us": round(p90 * 1e3, 2), "GBps": round(8.0 * n / (ms * 1e-3) / 1e9, 1),
             "Gelem_per_s": round(n / (ms * 1e-3) / 1e9, 2), "buffer_pairs": nbuf, "exact": bool(exact)}
        rows.append(r)
        log("sizes:", r)

    def exclusive_holds(xx, yy):
        return bool(yy[0] == 0) and bool(torch.equal(yy[1:] - yy[:-1], xx[:-1]))

    # 2^20 int32 in [0, 100): inclusive and exclusive, 64 buffer pairs (512 MiB)
    n1 = 1 << 20
    src = torch.from_numpy(workloads.uniform_i32(n1)).to(dev)
    pairs = [(src.clone(), torch.empty_like(src)) for _ in range(64)]
    for ex in (False, True):
        fns = [lambda p=p: scan.cumsum(p[0], exclusive=ex, out=p[1]) for p in pairs]
        t = _per_launch_ms(torch, fns, stream, 200)
        xx, yy = pairs[0]
        ok = exclusive_holds(xx, yy) if ex else inclusive_sum_holds(torch, xx, yy)
        row("int32 uniform[0,100) %s, n=2^20" % ("exclusive" if ex else "inclusive"), n1, t, ok, len(pairs))
    del pairs, src
    # 2^24 uint32: 8 buffer pairs (1 GiB)
    n2 = 1 << 24
    src = torch.from_numpy(workloads.full_u32(n2).view(np.int32)).to(dev)
    pairs = [(src.clone(), torch.empty_like(src)) for _ in range(8)]
    fns = [lambda p=p: scan.cumsum(p[0], out=p[1]) for p in pairs]
    t = _per_launch_ms(torch, fns, stream, 100)
    row("uint32 full-range inclusive, n=2^24", n2, t, inclusive_sum_holds(torch, *pairs[0]), len(pairs))
    del pairs, src
    # 2^28 in place on a copy of the bench input
    z = x.clone()
    scan.cumsum(z, out=z)
    torch.cuda.synchronize()
    ok = inclusive_sum_holds(torch, x, z)
    t = _per_launch_ms(torch, [lambda: scan.cumsum(z, out=z)], stream, 50)
    row("uint32 full-range inclusive in place, n=2^28", x.numel(), t, ok, 1)
    del z
    # 2^30 uint32
    n3 = 1 << 30
    big = torch.from_numpy(workloads.full_u32(n3).view(np.int32)).to(dev)
    out = torch.empty_like(big)
    t = _per_launch_ms(torch, [lambda: scan.cumsum(big, out=out)], stream, 20)
    row("uint32 full-range inclusive, n=2^30", n3, t, inclusive_sum_holds(torch, big, out), 1)
    del big, out
    return {"workload": "other sizes: int32 [0,100) seed 1001, uint32 full-range seed 1002; out of place unless "
                        "stated", "runs": rows}


def float32_run(scan, torch, workloads, stream):
    """Inclusive scan of 2^28 float32 normal(0,1); the input and result go to
    the CPU legs for the comparison with the oracle."""
    n = 1 << 28
    a = workloads.normal_f32(n)
    x = torch.from_numpy(a).to("cuda")
    y = torch.empty_like(x)
    ms, p10, p90 = _per_launch_ms(torch, [lambda: scan.cumsum(x, out=y)], stream, 50)
    res = {"workload": "inclusive scan, n=2^28 float32 normal(0,1) (seed 1003)",
           "scan_config": scan.selected_config(torch.float32, n), "us": round(ms * 1e3, 1),
           "p10_us": round(p10 * 1e3, 1), "p90_us": round(p90 * 1e3, 1),
           "GBps": round(8.0 * n / (ms * 1e-3) / 1e9, 1), "Gelem_per_s": round(n / (ms * 1e-3) / 1e9, 2)}
    log("float32:", res)
    got = y.cpu().numpy()
    del x, y
    return res, (a, got)


def float32_check(np, a, got):
    import oracle
    ref, ab = oracle.scan_f32(a)
    return bool(np.all(np.abs(got.astype(np.float64) - ref) <= oracle.f32_tolerance(ab)))


def autograd_run(scan, torch, workloads, stream):
    """The differentiable cumsum on 64 ragged rows: kernel times of the
    forward (segmented inclusive scan) and the backward (segmented reverse
    scan), and the time of one forward + backward through torch.autograd."""
    xs, gs, off = workloads.rows()
    n = xs.size
    x = torch.from_numpy(xs).to("cuda")
    g = torch.from_numpy(gs).to("cuda")
    offs = torch.from_numpy(off).to("cuda")
    y = torch.empty_like(x)
    gx = torch.empty_like(x)
    fwd = _per_launch_ms(torch, [lambda: scan.segmented_scan(x, offs, out=y)], stream, 50)
    bwd = _per_launch_ms(torch, [lambda: scan.cumsum_backward(g, offs, out=gx)], stream, 50)
    xr = x.clone().requires_grad_(True)

    def both():
        yy = scan.cumsum_autograd(xr, offs)
        yy.backward(g)
        return yy
    both()
    torch.cuda.synchronize()
    w = []
    for _ in range(10):
        xr.grad = None
        w0 = time.perf_counter()
        yy = both()
        torch.cuda.synchronize()
        w.append(time.perf_counter() - w0)
    w.sort()
    res = {"workload": "64 rows, lengths log-uniform in [2^10, 2^22] (n=%d), x and upstream grad normal(0,1) "
                       "(seed 1005)" % n,
           "forward_us": round(fwd[0] * 1e3, 1), "backward_us": round(bwd[0] * 1e3, 1),
           "forward_GBps": round(8.0 * n / (fwd[0] * 1e-3) / 1e9, 1),
           "backward_GBps": round(8.0 * n / (bwd[0] * 1e-3) / 1e9, 1),
           "autograd_fwd_bwd_wall_us": round(w[len(w) // 2] * 1e6, 1)}
    log("autograd:", res)
    data = (xs, gs, off, yy.detach().cpu().numpy(), xr.grad.cpu().numpy(), y.cpu().numpy(), gx.cpu().numpy())
    del x, g, offs, y, gx, xr
    return res, data


def autograd_check(np, xs, gs, off, y_ag, gx_ag, y_k, gx_k):
    """Forward and backward of the autograd rows against the oracle's
    per-row scan and suffix sums, within 2^-20 times the running sum of |.|."""
    import oracle
    ref, ab = oracle.segmented_f32(xs, off)
    tol = oracle.f32_tolerance(ab)
    fwd_ok = bool(np.all(np.abs(y_ag.astype(np.float64) - ref) <= tol)) and \
        bool(np.all(np.abs(y_k.astype(np.float64) - ref) <= tol))
    ref, ab = oracle.segmented_f32(gs, off, reverse=True)
    tol = oracle.f32_tolerance(ab)
    bwd_ok = bool(np.all(np.abs(gx_ag.astype(np.float64) - ref) <= tol)) and \
        bool(np.all(np.abs(gx_k.astype(np.float64) - ref) <= tol))
    return {"forward_within_bound_vs_oracle": fwd_ok, "backward_within_bound_vs_oracle": bwd_ok}


def compaction_run(scan, torch, x, y, stream):
    """Elements > 0 of the bench input read as int32, fused one-pass compaction."""
    n = x.numel()
    cnt = torch.empty(1, dtype=torch.int64, device=x.device)

    def run():
        scan.compact_into(x, y, cnt, "greater", 0)

    ms = _median_ms(torch, run, stream, 20)
    k = int(cnt.item())
    want = torch.masked_select(x, x > 0)
    ok = k == want.numel() and bool(torch.equal(y[:k], want))
    del want
    ms_torch = _sync_median_ms(torch, lambda: torch.masked_select(x, x > 0), stream, 5)
    moved = 4.0 * n + 4.0 * k
    res = {"workload": "keep x > 0 of the same n=2^%d input read as int32 (%d kept)" % (n.bit_length() - 1, k),
           "fused_us": round(ms * 1e3, 1), "GBps_moved": round(moved / (ms * 1e-3) / 1e9, 1),
           "bytes_moved": int(moved), "torch_masked_select_us": round(ms_torch * 1e3, 1),
           "speedup_vs_torch": round(ms_torch / ms, 2), "results_equal_torch_masked_select": bool(ok)}
    # two-way partition: every element written once (8 bytes per element)
    z = torch.empty_like(x)
    ms_p = _median_ms(torch, lambda: scan.partition_into(x, z, cnt, "greater", 0), stream, 20)
    kp = int(cnt.item())
    keep = x > 0
    ok_p = kp == k and bool(torch.equal(z[:kp], torch.masked_select(x, keep))) and \
        bool(torch.equal(z[kp:], torch.masked_select(x, ~keep).flip(0)))
    del z, keep
    res.update({"partition_us": round(ms_p * 1e3, 1), "partition_GBps": round(8.0 * n / (ms_p * 1e-3) / 1e9, 1),
                "partition_equal_torch": ok_p})
    log("compaction:", res)
    return res


def cpu_legs(args, np, a, got, alg_bytes, wide_f64):
    """The oracle on the host cores: the reported CPU baseline (repeated timed
    passes over the bench input), whose output is also the reference for the
    timed GPU result, for the paper's CPU scheme (context) and for the float64
    scan of the 'wide' object."""
    import oracle
    n = a.size
    reps, total, times, want = 0, 0.0, [], None
    while total < 10.0 and reps < 100:
        c0 = time.perf_counter()
        want = oracle.scan_int(a) if args.dtype == "u32" else oracle.scan_f32(a, with_abs=False)[0]
        dt = time.perf_counter() - c0
        times.append(dt)
        total += dt
        reps += 1
    times.sort()
    med = times[len(times) // 2]
    if args.dtype == "u32":
        equal = bool(np.array_equal(got.view(np.uint32), want))
    else:
        ref, ab = oracle.scan_f32(a)
        equal = bool(np.all(np.abs(got.astype(np.float64) - ref) <= np.ldexp(ab, -20)))
    cpu = {"value": round(alg_bytes / med / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
           "sample": "%d sequential passes over the same n=2^%d input (%.1f s), median pass %.3f s = %.3f Gelem/s"
                     % (reps, n.bit_length() - 1, total, med, n / med / 1e9),
           "gpu_result_equal_oracle" if args.dtype == "u32" else "gpu_result_within_bound": equal}
    log("cpu oracle:", cpu["value"], "GB/s; GPU result agrees:", equal)

    # the paper's multithreaded scheme on the host, for context
    cpu_ctx = None
    if args.dtype == "u32":
        import cpu_context
        threads = min(16, len(os.sched_getaffinity(0)))
        buf = np.empty_like(a)
        best, ok = None, True
        for part in (1 << 16, 1 << 18, 1 << 20):      # partition sizes tried (elements)
            times = []
            for _ in range(5):
                c0 = time.perf_counter()
                cpu_context.two_pass_scan_u32(a, threads, part, out=buf)
                times.append(time.perf_counter() - c0)
            ok = ok and bool(np.array_equal(buf, want))
            times.sort()
            med = times[len(times) // 2]
            if best is None or med < best[0]:
                best = (med, part)
        cpu_ctx = {"value": round(alg_bytes / best[0] / 1e9, 2), "unit": "GB/s", "cores": threads,
                   "kind": "paper two-pass Accumulate + Prefix Sum, best of 2^16 / 2^18 / 2^20-element "
                           "partitions (%d)" % best[1],
                   "equal_oracle": ok}
        log("cpu context:", cpu_ctx)

    # float64 result of the wide object against the double-double oracle
    f64_ok = None
    if wide_f64 is not None:
        f, yf = wide_f64
        ref, ab = oracle.scan_f64(f)
        depth = 8 * (-(-f.size // 32768)) + 128
        err = np.abs(yf - ref)
        f64_ok = {"within_bound": bool(np.all(err <= oracle.f64_tolerance(ab, depth))),
                  "max_err_over_sum_abs": float(np.max(err / np.maximum(ab, 1e-300)))}
    return cpu, cpu_ctx, f64_ok


def _median_ms(torch, fn, stream, reps):
    """Median kernel time of fn (which must not synchronise the host): each
    launch between its own pair of HIP events, all enqueued behind a GPU-side
    sleep so that no launch waits for the host between its events."""
    return _per_launch_ms(torch, [fn], stream, reps)[0]


def _sync_median_ms(torch, fn, stream, reps):
    """Median time of fn between HIP events with the host synchronised before
    every call: for calls that synchronise by themselves or are bound by
    host-side launches (their host cost belongs to the measurement)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def wide_runs(scan, torch, np, a, stream):
    """Inclusive scans of 2^28 uint64 and float64 elements (16 bytes moved per
    element).  uint64 is checked exactly on the GPU (y[0] = x[0], y[i] - y[i-1]
    = x[i] mod 2^64); the float64 input and result come back to the host for
    the CPU leg's comparison with the oracle."""
    n = a.size
    res = {"workload": "inclusive scan, n=2^%d, uint64 full-range (wrapping) and float64 normal(0,1) seed 1004"
                       % (n.bit_length() - 1)}
    a64 = (a.astype(np.uint64) << np.uint64(32)) | a[::-1].astype(np.uint64)
    x = torch.from_numpy(a64.view(np.int64)).to("cuda")
    del a64
    y = torch.empty_like(x)
    ms = _median_ms(torch, lambda: scan.cumsum(x, out=y), stream, 20)
    res["u64_us"] = round(ms * 1e3, 1)
    res["u64_GBps"] = round(16.0 * n / (ms * 1e-3) / 1e9, 1)
    res["u64_exact"] = inclusive_sum_holds(torch, x, y)
    log("wide u64: %.1f us" % (ms * 1e3))
    f = np.random.default_rng(1004).standard_normal(n)
    x = torch.from_numpy(f).to("cuda")
    y = torch.empty_like(x)
    ms = _median_ms(torch, lambda: scan.cumsum(x, out=y), stream, 20)
    res["f64_us"] = round(ms * 1e3, 1)
    res["f64_GBps"] = round(16.0 * n / (ms * 1e-3) / 1e9, 1)
    log("wide f64: %.1f us" % (ms * 1e3))
    yf = y.cpu().numpy()
    del x, y
    return res, (f, yf)


def inclusive_sum_holds(torch, x, y):
    """Exact test of an inclusive integer +-scan without a reference: y[0] =
    x[0] and y[i] - y[i-1] = x[i] in the tensors' wrapping arithmetic."""
    return bool(y[0] == x[0]) and bool(torch.equal(y[1:] - y[:-1], x[1:]))


def operator_runs(scan, torch, x, y, stream):
    """max / min / xor inclusive scans of the bench input read as int32.  Each
    result is checked exactly on the GPU by the recurrence that defines it:
    y[0] = x[0] and y[i] = y[i-1] (op) x[i] (signed compares)."""
    n = x.numel()
    res = {"workload": "inclusive scan of the same n=2^%d input read as int32 (signed compares)" % (n.bit_length() - 1)}
    ok = True
    combine = {"max": torch.maximum, "min": torch.minimum, "xor": torch.bitwise_xor}
    for op in ("max", "min", "xor"):
        def run():
            scan.cumsum(x, op=op, out=y)
        run()
        torch.cuda.synchronize()
        ok = ok and bool(y[0] == x[0]) and bool(torch.equal(y[1:], combine[op](y[:-1], x[1:])))
        ms = _median_ms(torch, run, stream, 20)
        res[op + "_us"] = round(ms * 1e3, 1)
        res[op + "_GBps"] = round(8.0 * n / (ms * 1e-3) / 1e9, 1)
        log("operator %s: %.1f us" % (op, ms * 1e3))
    res["results_exact"] = bool(ok)
    return res


def two_pass_comparison(scan, torch, x, y, single_ms, stream):
    """The paper's two-pass algorithms on the bench input, whole array and in
    partitions; each result must equal the single pass's output y."""
    n = x.numel()
    z = torch.empty_like(x)
    # the single pass's output again: the ceiling leg before this one reuses y
    scan.cumsum(x, out=y)
    torch.cuda.synchronize()
    rows, equal = [], True
    for method, floor in (("prefix_increment", 16), ("accumulate_prefix", 12)):
        for part in (0, 1 << 25, 1 << 24, 1 << 22):
            def run():
                scan.two_pass_cumsum(x, method, partition=part, out=z)
            run()
            torch.cuda.synchronize()
            equal = equal and bool(torch.equal(z, y))
            ms = _median_ms(torch, run, stream, 10)
            rows.append({"method": method, "partition": part, "us": round(ms * 1e3, 1),
                         "GBps_alg": round(8.0 * n / (ms * 1e-3) / 1e9, 1),
                         "min_bytes_per_elem": floor,
                         "GBps_min_traffic": round(floor * n / (ms * 1e-3) / 1e9, 1),
                         "time_vs_single_pass": round(ms / single_ms, 3)})
            log("two-pass:", rows[-1])
    return {"workload": "same input as the single pass; 16384-element tiles, one per workgroup; partition 0 = whole array",
            "single_pass_us": round(single_ms * 1e3, 1), "runs": rows, "results_equal": equal}


def segmented_comparison(scan, torch, np, workloads, dev, graphs=True):
    """Batched segmented scan (graph replay) vs one launch per segment; with
    graphs=False only the eager launches (the graph fields are null)."""
    import ctypes
    t0 = time.time()
    vals, off = workloads.segments()
    n = int(off[-1])
    S = off.size - 1
    x = torch.from_numpy(vals).to(dev)
    offs = torch.from_numpy(off).to(dev)
    y_b = torch.empty_like(x)
    y_l = torch.empty_like(x)
    y_g = torch.empty_like(x)
    log("segments ready: S=%d n=%d (%.1f s)" % (S, n, time.time() - t0))
    stream = torch.cuda.current_stream(dev)
    sptr = ctypes.c_void_p(stream.cuda_stream)

    g_batched = scan.SegmentedScanGraph(x, y_b, offs, exclusive=True) if graphs else None
    t_batched = _median_ms(torch, g_batched.launch, stream, 20) if graphs else None
    t_batched_eager = _median_ms(torch, lambda: scan.segmented_scan(x, offs, exclusive=True, out=y_b), stream, 20)
    # one launch per segment is bound by the host's launches: timed with them
    t_looped = _sync_median_ms(torch, lambda: scan.check(scan.lib.scan_segmented_looped(
        x.data_ptr(), y_l.data_ptr(), off.ctypes.data, S, scan.SCAN_I32, scan.SCAN_EXCLUSIVE, sptr)), stream, 5)
    g_looped = scan.LoopedScanGraph(x, y_g, off, exclusive=True) if graphs else None
    t_looped_graph = _median_ms(torch, g_looped.launch, stream, 5) if graphs else None
    if graphs:
        g_batched.launch()
    else:
        scan.segmented_scan(x, offs, exclusive=True, out=y_b)
    torch.cuda.synchronize()
    # an exclusive segmented +-scan is characterised exactly by y = 0 at every
    # segment start and y[i] = y[i-1] + x[i-1] elsewhere (mod 2^32)
    start = torch.zeros(n, dtype=torch.bool, device=dev)
    first = offs[:-1]
    start[first[first < n]] = True
    ok_b = bool((y_b[start] == 0).all()) and bool(((y_b[1:] - y_b[:-1] - x[:-1])[~start[1:]] == 0).all())
    ok_l = bool(torch.equal(y_l, y_b))
    ok_g = bool(torch.equal(y_g, y_b)) if graphs else True   # no graph result without graphs
    del start
    if graphs:
        g_batched.close()
        g_looped.close()
    alg = 8.0 * n + 8.0 * (S + 1)
    t_b = t_batched if graphs else t_batched_eager
    res = {
        "workload": "exclusive per-segment scan, S=%d, n=%d int32 Poisson(8), lengths log-uniform [1,2^20] (seed 1004)" % (S, n),
        "batched_graph_us": round(t_batched * 1e3, 1) if graphs else None,
        "batched_eager_us": round(t_batched_eager * 1e3, 1),
        "per_launch_eager_us": round(t_looped * 1e3, 1),
        "per_launch_graph_us": round(t_looped_graph * 1e3, 1) if graphs else None,
        "speedup_vs_eager": round(t_looped / t_b, 2),
        "speedup_vs_graph": round(t_looped_graph / t_b, 2) if graphs else None,
        "batched_GBps": round(alg / (t_b * 1e-3) / 1e9, 1),
        "results_equal": bool(ok_b and ok_l and ok_g),
    }
    log("segmented:", res)
    return res


if __name__ == "__main__":
    main()
