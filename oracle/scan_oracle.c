/*
 * Sequential CPU oracle for the prefix-sum hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or build flag
 * with the HIP kernels.
 *
 * What it computes (Introduction, definition of the scan):
 *   inclusive  out[i] = a[0] (+) a[1] (+) ... (+) a[i]
 *   exclusive  out[0] = identity, out[i] = a[0] (+) ... (+) a[i-1]
 * with (+) = addition, evaluated exactly as the basic algorithm the
 * Introduction describes: one sequential pass of additions over the input,
 * writing the running total.  Section 2 (thread-level parallelism) allows the
 * output to overwrite the input (in place); every routine here reads a[i]
 * before it writes out[i], so out == a is legal.
 *
 * Integer element types add in uint32_t, i.e. modulo 2^32 (the paper is silent
 * on overflow; wrap-around is the reading taken).  32-bit signed data is the
 * same bit pattern.  64-bit integers likewise add in uint64_t, modulo 2^64.
 * Float64 inputs are summed in double-double and rounded once (see
 * oracle_scan_f64): the reference is the definition's exact prefix sum to
 * within far less than one float64 rounding.  Float32 inputs are accumulated in float64 (the paper
 * notes that parallel float results may differ from the sequential ones; the
 * oracle therefore computes the sequential sum in a wider type and also
 * returns the running sum of absolute values, which sets the tolerance).
 *
 * Extensions that the paper does not define, read as follows:
 *   reverse   out[i] = a[i] (+) a[i+1] (+) ... (+) a[n-1]   (suffix scan; the
 *             exclusive form drops a[i]) -- the sequential pass runs from the
 *             last element down to the first;
 *   segmented offsets[0..S] (CSR form, offsets[0]=0, non-decreasing,
 *             offsets[S]=n) split the array into S independent segments;
 *             the running total restarts at the identity at each segment
 *             boundary, so each segment's result is the plain scan of that
 *             segment.  Empty segments are allowed.
 *
 * Build: gcc -O2 -std=c99 -shared -fPIC (no -ffast-math: the float64
 * additions must happen in program order).
 */
#include <stdint.h>
#include <math.h>
#include <string.h>

/* ---- other operators ---------------------------------------------------
 * The Introduction defines the scan for any associative operator with an
 * identity.  Besides +, the oracle computes three on 32-bit integers, by the
 * same sequential pass starting from the identity:
 *   op 1 max, op 2 min (signed when is_signed != 0, else unsigned), op 3 xor.
 * Identities: max INT32_MIN / 0, min INT32_MAX / UINT32_MAX, xor 0.  The
 * exclusive form writes the identity first.  */
static uint32_t op_identity(int op, int is_signed)
{
    switch (op) {
    case 1: return is_signed ? 0x80000000u : 0u;
    case 2: return is_signed ? 0x7FFFFFFFu : 0xFFFFFFFFu;
    default: return 0u;
    }
}

static uint32_t op_apply(int op, int is_signed, uint32_t acc, uint32_t x)
{
    switch (op) {
    case 1:
        if (is_signed) return (int32_t)x > (int32_t)acc ? x : acc;
        return x > acc ? x : acc;
    case 2:
        if (is_signed) return (int32_t)x < (int32_t)acc ? x : acc;
        return x < acc ? x : acc;
    default:
        return acc ^ x;
    }
}

void oracle_scan_op_u32(const uint32_t *a, uint32_t *out, int64_t n, int op,
                        int is_signed, int exclusive, int reverse)
{
    uint32_t acc = op_identity(op, is_signed);
    int64_t i = reverse ? n - 1 : 0;
    int64_t step = reverse ? -1 : 1;
    for (int64_t k = 0; k < n; ++k, i += step) {
        uint32_t x = a[i];
        if (exclusive) { out[i] = acc; acc = op_apply(op, is_signed, acc, x); }
        else           { acc = op_apply(op, is_signed, acc, x); out[i] = acc; }
    }
}

void oracle_segmented_op_u32(const uint32_t *a, uint32_t *out,
                             const int64_t *offsets, int64_t num_segments,
                             int op, int is_signed, int exclusive, int reverse)
{
    for (int64_t s = 0; s < num_segments; ++s) {
        int64_t lo = offsets[s], hi = offsets[s + 1];
        if (hi > lo)
            oracle_scan_op_u32(a + lo, out + lo, hi - lo, op, is_signed, exclusive, reverse);
    }
}

/* ---- flat scans -------------------------------------------------------- */

void oracle_scan_u32(const uint32_t *a, uint32_t *out, int64_t n,
                     int exclusive, int reverse)
{
    uint32_t acc = 0u;
    if (!reverse) {
        for (int64_t i = 0; i < n; ++i) {
            uint32_t x = a[i];
            if (exclusive) { out[i] = acc; acc += x; }
            else           { acc += x; out[i] = acc; }
        }
    } else {
        for (int64_t i = n - 1; i >= 0; --i) {
            uint32_t x = a[i];
            if (exclusive) { out[i] = acc; acc += x; }
            else           { acc += x; out[i] = acc; }
        }
    }
}

/* 64-bit integers: the same pass in uint64_t, modulo 2^64 (int64 data is the
 * same bit pattern); reverse runs it from the last element down. */
void oracle_scan_u64(const uint64_t *a, uint64_t *out, int64_t n, int exclusive, int reverse)
{
    uint64_t acc = 0u;
    int64_t i = reverse ? n - 1 : 0;
    const int64_t step = reverse ? -1 : 1;
    for (int64_t k = 0; k < n; ++k, i += step) {
        uint64_t x = a[i];
        if (exclusive) { out[i] = acc; acc += x; }
        else           { acc += x; out[i] = acc; }
    }
}

/* Float64 inputs: the prefix sums of the definition, rounded once to float64.
 * The running total is kept unevaluated as hi + lo (a double-double, about
 * 106 significant bits): each input is added to hi with Knuth's TwoSum, which
 * returns the rounded sum and its exact rounding error; the error joins lo
 * and the pair is renormalised (Dekker's Fast2Sum), so hi is the total
 * rounded to float64 and the accumulated error stays near n * 2^-106 *
 * sum|a|, far below one float64 rounding.  Non-finite inputs: once the
 * running total is infinite or NaN it is the plain IEEE sum (a NaN stays, an
 * infinity keeps its sign until the opposite one makes it NaN).  abs_out[i] (may be NULL): the
 * plain float64 running sum of |a|, the scale of the tolerance.  Reverse
 * runs the pass from the last element down (suffix sums). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *s = x;
    *e = (a - av) + (b - bv);
}

void oracle_scan_f64(const double *a, double *out, double *abs_out, int64_t n, int exclusive,
                     int reverse)
{
    double hi = 0.0, lo = 0.0, aacc = 0.0;
    int64_t i = reverse ? n - 1 : 0;
    const int64_t step = reverse ? -1 : 1;
    for (int64_t k = 0; k < n; ++k, i += step) {
        double x = a[i];
        if (exclusive) {
            out[i] = hi;
            if (abs_out) abs_out[i] = aacc;
        }
        double s, e;
        two_sum(hi, x, &s, &e);
        if (!isfinite(s)) {
            /* an infinite or NaN total has no rounding error to carry (and
             * TwoSum's inf - inf would turn +inf into NaN): the plain IEEE
             * sum, so NaN and infinities behave as in the definition */
            hi = s;
            lo = 0.0;
        } else {
            e += lo;
            hi = s + e;           /* Fast2Sum: |s| >= |e| after TwoSum */
            lo = e - (hi - s);
        }
        aacc += fabs(x);
        if (!exclusive) {
            out[i] = hi;
            if (abs_out) abs_out[i] = aacc;
        }
    }
}

/* out[i]: the sequential float64 prefix sum of the float32 inputs;
 * abs_out[i]: the same running sum over |a[j]| (may be NULL). */
void oracle_scan_f32_f64(const float *a, double *out, double *abs_out,
                         int64_t n, int exclusive, int reverse)
{
    double acc = 0.0, aacc = 0.0;
    int64_t i = reverse ? n - 1 : 0;
    int64_t step = reverse ? -1 : 1;
    for (int64_t k = 0; k < n; ++k, i += step) {
        double x = (double)a[i];
        if (exclusive) {
            out[i] = acc;
            if (abs_out) abs_out[i] = aacc;
            acc += x;
            aacc += fabs(x);
        } else {
            acc += x;
            aacc += fabs(x);
            out[i] = acc;
            if (abs_out) abs_out[i] = aacc;
        }
    }
}

/* ---- segmented scans --------------------------------------------------- */

void oracle_segmented_u32(const uint32_t *a, uint32_t *out,
                          const int64_t *offsets, int64_t num_segments,
                          int exclusive, int reverse)
{
    for (int64_t s = 0; s < num_segments; ++s) {
        int64_t lo = offsets[s], hi = offsets[s + 1];
        if (hi > lo)
            oracle_scan_u32(a + lo, out + lo, hi - lo, exclusive, reverse);
    }
}

void oracle_segmented_f32_f64(const float *a, double *out, double *abs_out,
                              const int64_t *offsets, int64_t num_segments,
                              int exclusive, int reverse)
{
    for (int64_t s = 0; s < num_segments; ++s) {
        int64_t lo = offsets[s], hi = offsets[s + 1];
        if (hi > lo)
            oracle_scan_f32_f64(a + lo, out + lo, abs_out ? abs_out + lo : 0,
                                hi - lo, exclusive, reverse);
    }
}

/* ---- stream compaction ---------------------------------------------------
 * The Introduction's partitioning / filtering use of the exclusive scan:
 * element i is kept when the predicate holds and then written to out[e_i],
 * e_i = the number of kept elements before i (the exclusive scan of the 0/1
 * selection).  Sequentially that is: append each kept element in order.
 * pred 0: keep x != 0 (its 32 bits); pred 1: keep x > thr compared as
 * int32 (dtype 0), uint32 (dtype 1) or float32 (dtype 2; NaN is never kept).
 * Returns the number kept; out[count..n) is not written. */
static int oracle_keep(uint32_t x, int pred, int dtype, uint32_t thr)
{
    if (pred == 0) return x != 0u;
    if (dtype == 0) return (int32_t)x > (int32_t)thr;
    if (dtype == 1) return x > thr;
    {
        float fx, ft;
        memcpy(&fx, &x, 4);
        memcpy(&ft, &thr, 4);
        return fx > ft;
    }
}

int64_t oracle_compact_u32(const uint32_t *a, uint32_t *out, int64_t n, int pred,
                           int dtype, uint32_t thr)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t x = a[i];
        if (oracle_keep(x, pred, dtype, thr)) out[k++] = x;
    }
    return k;
}

/* Two-way partition by the same predicate (the Introduction's partitioning
 * step: new offsets from a bitmap): element i goes to out[k] if kept, k being
 * the number kept before it, else to out[n-1-r], r being the number rejected
 * before it -- kept elements first in input order, the rest after them in
 * reverse input order.  Returns the number kept. */
int64_t oracle_partition_u32(const uint32_t *a, uint32_t *out, int64_t n, int pred,
                             int dtype, uint32_t thr)
{
    int64_t k = 0, r = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t x = a[i];
        if (oracle_keep(x, pred, dtype, thr)) out[k++] = x;
        else out[n - 1 - r++] = x;
    }
    return k;
}
