/*
 * mi355scan -- single-pass prefix sums (scans) on AMD Instinct MI355X (gfx950).
 *
 * The operation is the scan of the paper's Introduction: for an input
 * a[0..n-1] and the operator +, the inclusive scan writes
 *     out[i] = a[0] + a[1] + ... + a[i]
 * and the exclusive scan writes the identity (0) first and drops the last
 * inclusive value:  out[0] = 0, out[i] = a[0] + ... + a[i-1].
 * Section 2 (thread-level parallelism) allows the result to replace the input:
 * in == out is legal everywhere below (in place) except for scan_partition;
 * any other overlap is an error.
 *
 * The GPU method is the device-scale form of the paper's cache-friendly
 * two-pass scheme (Section 2.2): every tile of the input is loaded once into
 * registers, scanned there (the wavefront scan is the 64-lane analogue of the
 * horizontal in-register scan of Section 3.1), and written once, while the
 * carry between tiles travels through a chain of per-tile status words in
 * which each tile waits only on its predecessors (the adjacent-only
 * synchronisation that Section 2.2.1 suggests in place of a central barrier).
 * HBM traffic is therefore the two-words-per-element floor: 8 bytes per
 * element for every 32-bit scan (16 for 64-bit elements), plus 8 bytes per
 * tile of status (16 for 64-bit elements).
 *
 * Conventions for every function:
 *  - Pointers named in/out/grad_* and offsets are DEVICE pointers owned by the
 *    caller; they must stay valid until the work enqueued on `stream`
 *    completes.  32-bit elements need 4-byte alignment, offsets 8-byte
 *    alignment; 16-byte aligned buffers take the vector fast path
 *    automatically.  64-bit elements need 16-byte aligned buffers.
 *  - All functions are asynchronous on `stream` (a hipStream_t; 0 = the null
 *    stream) and do not synchronise the host, except where a workspace has to
 *    grow (see scan_reserve).
 *  - Argument errors are detected on the host and returned before anything is
 *    enqueued.  n == 0 is a successful no-op.  Malformed offsets CONTENTS
 *    (device data) are not checked: the kernels never read or write outside
 *    in[0..n), out[0..n), offsets[0..S], but the results are then unspecified.
 *  - No function aborts or throws across the ABI; a failing HIP call is
 *    reported as SCAN_ERROR_LAUNCH / SCAN_ERROR_OUT_OF_MEMORY and its hipError_t
 *    is kept for scan_last_hip_error().
 *  - Device-side waits (a tile waiting for its predecessors' status words)
 *    are bounded (scan_set_spin_limit).  A wait that gives up lets the kernel
 *    finish and raises the error word of the stream (or library graph) it ran
 *    on; that call's results are invalid.  The word lives in host memory and
 *    is read without synchronising: the next call on the same stream (the
 *    next scan_graph_launch of the same graph) that finds it raised returns
 *    SCAN_ERROR_TIMEOUT, clears it and enqueues nothing.  A call made while
 *    the failing kernel is still running cannot see it yet; the first one
 *    after it has finished does (scan_check_device_error waits for that).
 *  - Integer scans wrap modulo 2^32 (2^64 for 64-bit elements); signed and
 *    unsigned types of one width give identical bits.
 *  - float32 scans: the result is within 2^-20 * sum_{j<=i} |a_j| of the exact
 *    prefix sum (sum_{j<i} for exclusive).  The paper notes that parallel float
 *    sums may differ slightly from sequential ones; this library fixes the
 *    summation order per tuning configuration, so repeated runs give identical
 *    bits.
 *  - Concurrency: each stream gets its own workspace; calls on one stream run
 *    in stream order.  Two host threads may call concurrently on different
 *    streams.
 */
#ifndef MI355SCAN_H
#define MI355SCAN_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCAN_SUCCESS = 0,
    SCAN_ERROR_INVALID_VALUE = 1,   /* bad pointer, size, alignment, flag or dtype */
    SCAN_ERROR_OVERLAP = 2,         /* in and out overlap without being equal */
    SCAN_ERROR_OUT_OF_MEMORY = 3,   /* workspace allocation failed */
    SCAN_ERROR_LAUNCH = 4,          /* a HIP call failed (see scan_last_hip_error) */
    SCAN_ERROR_NOT_SUPPORTED = 5,   /* no gfx950 device, or unsupported combination */
    SCAN_ERROR_CAPTURE = 6,         /* would allocate while the stream is being captured */
    SCAN_ERROR_TIMEOUT = 7          /* a device-side wait hit its spin limit */
} scan_status_t;

/* SCAN_I64 / SCAN_U64: 64-bit integer sums (wrapping modulo 2^64, the same
 * bits for both); SCAN_F64: float64 sums.  scan_flat only: see scan_flat. */
typedef enum {
    SCAN_I32 = 0, SCAN_U32 = 1, SCAN_F32 = 2, SCAN_I64 = 3, SCAN_U64 = 4, SCAN_F64 = 5
} scan_dtype_t;

/* Flag bits. */
#define SCAN_EXCLUSIVE 0x1u  /* exclusive scan (identity first)              */
#define SCAN_REVERSE   0x2u  /* suffix scan: out[i] = a[i] + ... + a[n-1]     */
/* Operator field (bits 2-3).  The Introduction defines the scan for any
 * associative operator with an identity; besides + (the default, field 0)
 * the integer dtypes take:
 *   SCAN_OP_MAX  maximum  (identity INT32_MIN for i32, 0 for u32)
 *   SCAN_OP_MIN  minimum  (identity INT32_MAX for i32, UINT32_MAX for u32)
 *   SCAN_OP_XOR  bitwise exclusive or (identity 0)
 * i32 compares as signed, u32 as unsigned; the exclusive first element is
 * the identity.  Valid for flat, segmented, looped and graph calls; float32
 * with an operator other than +, SCAN_REVERSE with SCAN_OP_MIN, and
 * SCAN_REVERSE with SCAN_OP_MAX on i32 return SCAN_ERROR_NOT_SUPPORTED, and so
 * do the two-pass scans with any operator other than +. */
#define SCAN_OP_MAX    0x4u
#define SCAN_OP_MIN    0x8u
#define SCAN_OP_XOR    0xCu

/* ---- flat scans (Introduction: definition; Section 2: in place or not) ----
 * in, out: device arrays of n elements (in == out allowed).  n >= 0. */
scan_status_t scan_inclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t stream);
scan_status_t scan_inclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t stream);
scan_status_t scan_inclusive_f32(const float *in, float *out, int64_t n, hipStream_t stream);
scan_status_t scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t stream);
scan_status_t scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t stream);
scan_status_t scan_exclusive_f32(const float *in, float *out, int64_t n, hipStream_t stream);

/* General flat scan: any dtype, flags = SCAN_EXCLUSIVE | SCAN_REVERSE, plus
 * an operator (SCAN_OP_*) for i32 / u32.
 * SCAN_I64 / SCAN_U64 / SCAN_F64 (the Introduction's scan with + on 64-bit
 * elements, e.g. offsets past 2^32 or float64 data): in and out must be
 * 16-byte aligned (SCAN_ERROR_INVALID_VALUE otherwise), flags SCAN_EXCLUSIVE
 * and SCAN_REVERSE (an operator: SCAN_ERROR_NOT_SUPPORTED).  Integers are
 * bit-exact, wrapping modulo 2^64; a float64 result is a sum of the same
 * inputs in another association, within (8 * tiles + 128) * 2^-53 times the
 * running sum of |a| of the exact prefix sum (tiles = ceil(n / 32768); the
 * depth of the addition tree, see the 64-bit kernel).  The other entry points
 * return SCAN_ERROR_NOT_SUPPORTED for these dtypes.  Uses the stream's
 * workspace (two status words per 32768-element tile). */
scan_status_t scan_flat(const void *in, void *out, int64_t n, scan_dtype_t dtype,
                        uint32_t flags, hipStream_t stream);

/* ---- allocation-free flat scan ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Computes
 * exactly what scan_flat computes for the 32-bit dtypes (SCAN_I32 / SCAN_U32
 * / SCAN_F32, every flag and operator scan_flat accepts for them), but its
 * tile status words, counters and error word live in a fixed array of the
 * library in device memory (one copy per device, 540,736 bytes, zero when
 * the library loads, held until the process ends) instead of a stream
 * workspace, and the call makes no allocation of any kind (no hipMalloc,
 * hipFree or hipHostMalloc; the first call on a device only looks up that
 * device's copy of the array).  Arguments and results are scan_flat's.
 * Limit: 32768 tiles, i.e. n <= 3,221,225,472 when in and out are 16-byte
 * aligned (98,304-element tiles at most) and n <= 268,435,456 otherwise
 * (8,192-element tiles); a larger n returns SCAN_ERROR_INVALID_VALUE, a
 * 64-bit dtype SCAN_ERROR_NOT_SUPPORTED, both before anything is enqueued.
 * Every call on one device shares that device's array, and each call leaves
 * it clean for the next: calls whose kernels overlap in time on one device
 * (two streams, two host threads) race and give wrong results, so keep them
 * on one stream.  A device-side wait that gives up raises the array's error
 * word; scan_check_device_error (with that device current, any stream)
 * reports and clears it.  Graphs captured from these calls stay valid for
 * the life of the process. */
scan_status_t scan_flat_noalloc(const void *in, void *out, int64_t n, scan_dtype_t dtype,
                                uint32_t flags, hipStream_t stream);

/* ---- batched segmented scan (one persistent launch) ----
 * Scans num_segments independent segments of one concatenated array: segment
 * s covers in[offsets[s] .. offsets[s+1]), and each segment's result is the
 * flat scan of that segment alone (the running total restarts at every
 * segment start; exclusive results are 0 at a segment's first element).
 * This is the histogram-to-offsets use of the Introduction done for many
 * histograms at once.
 * offsets: device int64[num_segments + 1], offsets[0] = 0, non-decreasing,
 * offsets[num_segments] = n; empty segments allowed.  num_segments >= 1 when
 * n > 0.  Enqueues two kernels (a tile-to-segment map and the scan). */
scan_status_t scan_segmented_batch(const void *in, void *out, const int64_t *offsets,
                                   int32_t num_segments, int64_t n, scan_dtype_t dtype,
                                   uint32_t flags, hipStream_t stream);

/* ---- two-pass scans (comparison with the single pass) ----
 * The multithreaded two-pass algorithms of Section 2.1 at device scale, a
 * workgroup in the role of the paper's thread and a 16384-element tile in the
 * role of its partition:
 *  SCAN_TWO_PASS_PREFIX_INCREMENT  ("Prefix Sum + Increment") pass 1 scans
 *      every tile and writes it, keeping its total; pass 2 adds to every tile
 *      the sum of the totals before it.  HBM traffic 16 bytes per element.
 *  SCAN_TWO_PASS_ACCUMULATE_PREFIX ("Accumulate + Prefix Sum") pass 1 only
 *      adds up every tile; pass 2 scans every tile starting from the sum of
 *      the totals before it.  HBM traffic 12 bytes per element.
 * Between the passes one workgroup scans the tile totals.
 * partition: elements per partition of the cache-friendly scheme of Section
 * 2.2 (rounded up to whole tiles): both passes run on one partition before
 * the next starts, so pass 2 may find pass 1's data in the caches; 0 = one
 * partition holding everything.  Each partition costs three launches.
 * flags: SCAN_EXCLUSIVE only; SCAN_REVERSE returns SCAN_ERROR_NOT_SUPPORTED.
 * in == out allowed.  Results: the same contract as scan_flat (bit-exact for
 * integers, the float32 bound).  Uses the stream's workspace. */
#define SCAN_TWO_PASS_PREFIX_INCREMENT  0
#define SCAN_TWO_PASS_ACCUMULATE_PREFIX 1
scan_status_t scan_two_pass(const void *in, void *out, int64_t n, scan_dtype_t dtype,
                            uint32_t flags, int32_t method, int64_t partition,
                            hipStream_t stream);

/* ---- stream compaction fused with the exclusive scan ----
 * The Introduction's use of prefix sums as new index values (partitioning,
 * parallel filtering): out receives, in order, the elements of in[0..n) that
 * the predicate keeps -- element i goes to out[e_i], e_i = the number of kept
 * elements before i, i.e. the exclusive scan of the 0/1 selection -- and
 * *count the number kept.  One pass over in; out[*count .. n) is left as it
 * was.
 * predicate: SCAN_PRED_NONZERO keeps elements whose 32 bits are not all zero
 *   (threshold ignored); SCAN_PRED_GREATER keeps x > threshold, compared as
 *   int32, uint32 or float32 by dtype (threshold holds the value's bits; a NaN
 *   is never kept).
 * in, out: n elements (in == out allowed); count: device int64, 8-byte
 * aligned, written by the kernel.  n < 2^32.  Uses the stream's workspace. */
#define SCAN_PRED_NONZERO 0
#define SCAN_PRED_GREATER 1
scan_status_t scan_compact(const void *in, void *out, int64_t n, scan_dtype_t dtype,
                           int32_t predicate, uint32_t threshold, int64_t *count,
                           hipStream_t stream);

/* ---- two-way partition (one pass) ----
 * The partitioning step of the Introduction (new offsets from a bitmap) with
 * both sides kept: element i of in[0..n) goes to out[e_i] when the predicate
 * keeps it (e_i = the number kept before i, as in scan_compact) and otherwise
 * to out[n-1-r_i], r_i = i - e_i being the number rejected before it.  The
 * kept elements fill out[0 .. *count) in input order, the rejected ones
 * out[*count .. n) in reverse input order; every element is written once.
 * predicate, threshold, count, n: as for scan_compact.  in and out must not
 * overlap, in == out included (SCAN_ERROR_OVERLAP): rejected elements are
 * written ahead of the data still to be read.  Uses the stream's workspace. */
scan_status_t scan_partition(const void *in, void *out, int64_t n, scan_dtype_t dtype,
                             int32_t predicate, uint32_t threshold, int64_t *count,
                             hipStream_t stream);

/* ---- float32 cumsum backward ----
 * For y = inclusive cumsum of x (per segment if offsets != NULL), the
 * gradient is the suffix sum of the upstream gradient:
 *     grad_in[i] = sum_{j >= i, j in the same segment} grad_out[j].
 * offsets may be NULL (one segment of length n; num_segments ignored).
 * grad_in == grad_out is allowed. */
scan_status_t scan_f32_backward(const float *grad_out, float *grad_in, int64_t n,
                                const int64_t *offsets, int32_t num_segments,
                                hipStream_t stream);

/* ---- workspace ----
 * Each stream owns a workspace (tile status words and counters) that is
 * allocated on first use and grown when a larger n arrives; growing
 * synchronises the stream and is refused during stream capture (returns
 * SCAN_ERROR_CAPTURE).  Call scan_reserve(max_n) before capturing library
 * calls into a graph of your own.  Growing never frees the allocation it
 * replaces: a graph captured from calls on this stream keeps using it and
 * stays valid (and exact) after later, larger eager calls.  Replays of such
 * graphs, and eager calls on the stream, must not overlap in time.
 * The workspace keeps itself clean between launches (no reset kernel or
 * memset is needed per call). */
scan_status_t scan_reserve(int64_t max_n, hipStream_t stream);
/* Frees every workspace the stream has used (current and outgrown) and its
 * error word; synchronises the stream.  Graphs captured from this stream's
 * calls become invalid: destroy them first. */
scan_status_t scan_release(hipStream_t stream);

/* ---- graphs ----
 * Capture a batched segmented scan (both kernels) into a hipGraph with its own
 * workspace; replay it with scan_graph_launch (on any stream; replays of one
 * graph must not overlap in time).  The buffers are bound at creation: the
 * caller may change their contents between replays but not their addresses. */
scan_status_t scan_segmented_graph_create(const void *in, void *out, const int64_t *offsets,
                                          int32_t num_segments, int64_t n, scan_dtype_t dtype,
                                          uint32_t flags, hipStream_t stream, void **graph);
/* Comparator: one flat-scan launch per segment (host_offsets: HOST int64[S+1]),
 * captured into one graph; replay with scan_graph_launch. */
scan_status_t scan_looped_graph_create(const void *in, void *out, const int64_t *host_offsets,
                                       int32_t num_segments, scan_dtype_t dtype,
                                       uint32_t flags, hipStream_t stream, void **graph);
/* Replays a graph; returns SCAN_ERROR_TIMEOUT (and replays nothing) when an
 * earlier replay of this graph gave up a device-side wait. */
scan_status_t scan_graph_launch(void *graph, hipStream_t stream);
/* Reads and clears the graph's error word without synchronising: call it
 * after the replay has finished (e.g. after synchronising its stream).
 * SCAN_SUCCESS or SCAN_ERROR_TIMEOUT. */
scan_status_t scan_graph_check_device_error(void *graph);
scan_status_t scan_graph_destroy(void *graph);

/* Comparator: one flat-scan launch per segment, enqueued eagerly from the
 * host (host_offsets: HOST int64[S+1]).  Results equal scan_segmented_batch. */
scan_status_t scan_segmented_looped(const void *in, void *out, const int64_t *host_offsets,
                                    int32_t num_segments, scan_dtype_t dtype,
                                    uint32_t flags, hipStream_t stream);

/* ---- tuning ----
 * Kernel configurations are numbered 0 .. scan_num_configs()-1; each fixes the
 * workgroup size, the elements per thread (tile = threads * items; the tile is
 * the GPU counterpart of the paper's cache-sized partition, Section 2.2, whose
 * size the paper tunes in Section 4.2.4), non-temporal memory hints and
 * how tiles are assigned to workgroups.  A tuning table maps (dtype, flags, segmented, log2 n bucket)
 * to a configuration; built-in defaults can be replaced from a JSON file. */
int32_t       scan_num_configs(void);
/* Describes configuration `config` (any output pointer may be NULL):
 *  block, items: threads per workgroup and elements per thread (tile =
 *    block * items elements);
 *  nontemporal: 1 if tile loads and stores carry the non-temporal hint;
 *  mode: how tiles reach workgroups:
 *       0 = one tile per workgroup, tile numbers from a device counter;
 *       1 = resident grid taking tiles from the counter;
 *       2 = tile number = workgroup index (no counter; relies on workgroups
 *           being dispatched in index order, bounded by the spin limit);
 *       4 = static round robin over a cooperatively launched resident grid;
 *  per_cu: resident-grid modes: workgroups per CU (0 = as many as fit);
 *  cu_pct: resident-grid modes: percent of the CUs the grid covers.
 * Inputs or outputs that are not 16-byte aligned always run a dword-access
 * kernel (256 x 32, mode 1) whatever the configuration. */
scan_status_t scan_config_info(int32_t config, int32_t *block, int32_t *items,
                               int32_t *nontemporal, int32_t *mode, int32_t *per_cu,
                               int32_t *cu_pct);
/* Force a configuration for subsequent calls (-1 = use the tuning table). */
scan_status_t scan_force_config(int32_t config);
/* Configuration the table selects for a call of this shape. */
int32_t       scan_selected_config(scan_dtype_t dtype, uint32_t flags, int32_t segmented, int64_t n);
/* Time every configuration on the caller's buffers (in, out: n elements;
 * offsets/num_segments for segmented, else NULL/0), store the fastest in the
 * table for n's bucket and return it in *best (may be NULL).  Synchronises. */
scan_status_t scan_autotune(const void *in, void *out, int64_t n, const int64_t *offsets,
                            int32_t num_segments, scan_dtype_t dtype, uint32_t flags,
                            int32_t reps, hipStream_t stream, int32_t *best);
scan_status_t scan_tune_save(const char *path);
scan_status_t scan_tune_load(const char *path);

/* ---- diagnostics ---- */
const char   *scan_status_string(scan_status_t status);
int32_t       scan_last_hip_error(void);
/* Spin limit for device-side waits (sleeping polls; 0 restores the default
 * of 2^16, about 0.1 s).  A wait that exceeds it gives up, raises the error
 * word of the stream or graph and lets the kernel finish (the results of that
 * call are then invalid).  Applies to launches enqueued (or graphs created)
 * after the call. */
scan_status_t scan_set_spin_limit(uint32_t limit);
/* Streaming ceiling of the scan's memory access pattern (measurement, not a
 * scan): out[i] = in[i] + 1 modulo 2^32 for n 32-bit elements, with the tile
 * shape, grid, tile counter, 128-bit buffer accesses, cache policy and
 * store/load hand-off of scan configuration `config` (scan_config_info;
 * counter modes 0 and 1 only, others return SCAN_ERROR_NOT_SUPPORTED), but
 * without the in-register scan and the look-back.  It moves the scan's 8
 * bytes per element, the two-words-per-element floor that the partitioned
 * scan of Section 2.2 reaches, so its time is the floor of the scan kernel of
 * that shape.  in and out must be 16-byte aligned (SCAN_ERROR_INVALID_VALUE
 * otherwise); in == out is allowed.  Uses the stream's workspace (tile
 * counter). */
scan_status_t scan_stream_ceiling(const void *in, void *out, int64_t n, int32_t config, hipStream_t stream);

/* Synchronise `stream`, read and clear its error word, and the error word of
 * the current device's scan_flat_noalloc array once a call has used it:
 * SCAN_SUCCESS, or SCAN_ERROR_TIMEOUT if either was raised. */
scan_status_t scan_check_device_error(hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MI355SCAN_H */
