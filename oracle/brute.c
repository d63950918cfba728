/*
 * Oracle for exact online string matching: direct comparison at every
 * window start.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The product path never
 * links, loads or calls it, and it shares no code, header or table with
 * the HIP path.
 *
 * Definition followed (problem statement, Section 1, and the string
 * notation of Section 2): the occurrences of a pattern x of length m in a
 * text y of length n are the positions t with 0 <= t <= n - m such that
 * y[t + k] = x[k] for every 0 <= k < m. Characters are compared as unsigned
 * bytes. Every such t is reported, overlapping ones included, in ascending
 * order.
 *
 * Threads only split the range of window starts into consecutive blocks;
 * each block is scanned with the same plain loop and the per-block lists are
 * concatenated in block order, so the result does not depend on the number
 * of threads.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const unsigned char *x;
    const unsigned char *y;
    int64_t m;
    int64_t lo, hi;      /* window starts lo <= t < hi */
    int64_t *pos;        /* found starts, ascending */
    int64_t count;
    int64_t capacity;
    int failed;
} block_job;

static void *scan_block(void *arg)
{
    block_job *job = (block_job *)arg;
    for (int64_t t = job->lo; t < job->hi; ++t) {
        if (memcmp(job->y + t, job->x, (size_t)job->m) != 0)
            continue;
        if (job->count == job->capacity) {
            int64_t grown = job->capacity ? 2 * job->capacity : 1024;
            int64_t *p = (int64_t *)realloc(job->pos, (size_t)grown * sizeof(int64_t));
            if (!p) {
                job->failed = 1;
                return NULL;
            }
            job->pos = p;
            job->capacity = grown;
        }
        job->pos[job->count++] = t;
    }
    return NULL;
}

/*
 * All occurrences of x[0..m-1] in y[0..n-1].
 * Writes the first min(count, cap) start positions, ascending, to out
 * (out may be NULL when cap is 0) and returns count, the true total.
 * Returns -1 on bad arguments (m < 1, n < 0, threads < 1) and -2 when
 * memory runs out.
 */
int64_t oracle_occurrences(const unsigned char *x, int64_t m,
                           const unsigned char *y, int64_t n,
                           int64_t *out, int64_t cap, int threads)
{
    if (m < 1 || n < 0 || threads < 1 || cap < 0)
        return -1;
    if (n < m)
        return 0;
    int64_t starts = n - m + 1;
    if (threads > starts)
        threads = (int)starts;

    block_job *jobs = (block_job *)calloc((size_t)threads, sizeof(block_job));
    pthread_t *tids = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tids) {
        free(jobs);
        free(tids);
        return -2;
    }
    for (int b = 0; b < threads; ++b) {
        jobs[b].x = x;
        jobs[b].y = y;
        jobs[b].m = m;
        jobs[b].lo = starts * b / threads;
        jobs[b].hi = starts * (b + 1) / threads;
    }
    int spawned = 0;
    for (int b = 1; b < threads; ++b) {
        if (pthread_create(&tids[b], NULL, scan_block, &jobs[b]) != 0)
            break;
        spawned = b;
    }
    scan_block(&jobs[0]);
    for (int b = 1; b <= spawned; ++b)
        pthread_join(tids[b], NULL);
    /* blocks whose thread could not be started run here */
    for (int b = spawned + 1; b < threads; ++b)
        scan_block(&jobs[b]);

    int64_t total = 0;
    int failed = 0;
    for (int b = 0; b < threads; ++b) {
        failed |= jobs[b].failed;
        for (int64_t k = 0; k < jobs[b].count; ++k, ++total)
            if (total < cap)
                out[total] = jobs[b].pos[k];
        free(jobs[b].pos);
    }
    free(jobs);
    free(tids);
    return failed ? -2 : total;
}

/* Number of occurrences only (same definition, nothing written). */
int64_t oracle_count(const unsigned char *x, int64_t m,
                     const unsigned char *y, int64_t n, int threads)
{
    return oracle_occurrences(x, m, y, n, NULL, 0, threads);
}

/* Whether x occurs at window start t of y: the definition for one t. */
int oracle_matches_at(const unsigned char *x, int64_t m,
                      const unsigned char *y, int64_t n, int64_t t)
{
    if (m < 1 || t < 0 || t > n - m)
        return 0;
    return memcmp(y + t, x, (size_t)m) == 0;
}
