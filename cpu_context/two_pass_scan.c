/*
 * The paper's multithreaded scan on the host CPU, for context beside the GPU
 * path and the sequential oracle (not a fallback: nothing in the GPU library
 * calls it).
 *
 * Scheme (Section 2.1, "Accumulate + Prefix Sum", with the cache-friendly
 * partitioning of Section 2.2, the paper's Scalar2-P): the array is processed
 * in iterations of `threads` partitions of `partition` elements each.  In
 * iteration k thread m first adds up its partition into sums_{k%2}[m]
 * (pass 1, no writes), all threads meet at one counting barrier, then thread
 * m scans its partition -- still in its cache -- starting from the total of
 * everything before it: the running total of the earlier iterations plus
 * sums_{k%2}[0..m-1] (pass 2).  There is no barrier after pass 2: the two
 * sums arrays alternate, and the barrier of iteration k+1 keeps iteration k+2
 * from overwriting sums_{k%2} while a thread still reads it (Section 2.2.1).
 * Every thread keeps its own copy of the running total.  Integers wrap
 * modulo 2^32.
 *
 * Build: gcc -O3 -std=c11 -pthread -shared -fPIC.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    atomic_int count;
    atomic_int phase;
    int nthreads;
} barrier_t;

/* Reusable counting barrier: the last thread to arrive resets the count and
 * advances the phase; the others spin on the phase. */
static void barrier_wait(barrier_t *b)
{
    const int ph = atomic_load_explicit(&b->phase, memory_order_acquire);
    if (atomic_fetch_add_explicit(&b->count, 1, memory_order_acq_rel) == b->nthreads - 1) {
        atomic_store_explicit(&b->count, 0, memory_order_relaxed);
        atomic_store_explicit(&b->phase, ph + 1, memory_order_release);
    } else {
        while (atomic_load_explicit(&b->phase, memory_order_acquire) == ph) {
        }
    }
}

typedef struct {
    const uint32_t *in;
    uint32_t *out;
    int64_t n;
    int64_t partition;
    int threads;
    uint32_t *sums;      /* [2][threads] */
    barrier_t *bar;
    atomic_int go;       /* 0 wait, 1 run, -1 give up (a thread did not start) */
} shared_t;

typedef struct {
    shared_t *s;
    int m;
} arg_t;

static void *worker(void *p)
{
    const arg_t *a = (const arg_t *)p;
    shared_t *s = a->s;
    int g;
    while ((g = atomic_load_explicit(&s->go, memory_order_acquire)) == 0) {
    }
    if (g < 0) return NULL;
    const int m = a->m, T = s->threads;
    const int64_t P = s->partition, round = P * T;
    uint32_t running = 0u;
    for (int64_t base = 0, k = 0; base < s->n; base += round, ++k) {
        uint32_t *sums = s->sums + (k & 1) * T;
        const int64_t lo = base + m * P < s->n ? base + m * P : s->n;
        const int64_t hi = lo + P < s->n ? lo + P : s->n;
        /* pass 1: accumulate the partition */
        uint32_t acc = 0u;
        for (int64_t i = lo; i < hi; ++i) acc += s->in[i];
        sums[m] = acc;
        barrier_wait(s->bar);
        /* pass 2: scan the partition from the total before it */
        uint32_t off = running, all = running;
        for (int i = 0; i < T; ++i) {
            if (i < m) off += sums[i];
            all += sums[i];
        }
        running = all;
        for (int64_t i = lo; i < hi; ++i) {
            off += s->in[i];
            s->out[i] = off;
        }
    }
    return NULL;
}

/* Inclusive uint32 scan of in[0..n) into out (in == out allowed) with
 * `threads` threads and partitions of `partition` elements.  Returns 0, or -1
 * if a thread could not be started or memory could not be allocated. */
int cpu_two_pass_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, int threads, int64_t partition)
{
    if (n <= 0) return 0;
    if (threads < 1) threads = 1;
    if (partition < 1) partition = 1;
    barrier_t bar;
    atomic_init(&bar.count, 0);
    atomic_init(&bar.phase, 0);
    bar.nthreads = threads;
    uint32_t *sums = (uint32_t *)calloc(2 * (size_t)threads, sizeof(uint32_t));
    pthread_t *tid = (pthread_t *)malloc((size_t)threads * sizeof(pthread_t));
    arg_t *args = (arg_t *)malloc((size_t)threads * sizeof(arg_t));
    if (!sums || !tid || !args) {
        free(sums);
        free(tid);
        free(args);
        return -1;
    }
    shared_t s = {in, out, n, partition, threads, sums, &bar, 0};
    atomic_init(&s.go, 0);
    int started = 0, rc = 0;
    for (int m = 1; m < threads; ++m) {
        args[m].s = &s;
        args[m].m = m;
        if (pthread_create(&tid[m], NULL, worker, &args[m]) != 0) {
            rc = -1;
            break;
        }
        ++started;
    }
    atomic_store_explicit(&s.go, rc == 0 ? 1 : -1, memory_order_release);
    if (rc == 0) {
        args[0].s = &s;
        args[0].m = 0;
        worker(&args[0]);
    }
    for (int m = 1; m <= started; ++m) pthread_join(tid[m], NULL);
    free(sums);
    free(tid);
    free(args);
    return rc;
}
