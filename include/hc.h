/*
 * hc.h -- C ABI of libhc: the searching phase of the Hash Chain (HC) exact
 * string-matching algorithm (Palmer, Faro, Scafiti, "Efficient Online String
 * Matching through Linked Weak Factors") on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 1; notation of Section 2): given a pattern x[0..m-1] and a
 * text y[0..n-1] over bytes, report every start t, 0 <= t <= n-m, with
 * y[t..t+m-1] = x. Characters are unsigned 8-bit values. Results are
 * ascending int64 start positions, overlapping occurrences included, no
 * duplicates. The set never depends on q, alpha, w or the launch shape.
 *
 * Conventions for every call:
 *   - Nothing aborts or throws across this boundary; every call returns an
 *     hc_status (hc_strerror() names it).
 *   - "d_" pointers are device pointers on the current HIP device; all other
 *     pointers are host pointers.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is ordered on that stream; calls on one stream serialise,
 *     calls on different streams may run concurrently. Several host threads
 *     may enqueue searches on the same stream: each call's kernels are
 *     enqueued together, never interleaved with another call's.
 *   - The caller owns every text and output buffer and keeps device buffers
 *     alive until the stream work that uses them has finished.
 *   - Text lengths are limited to n <= 2^32 - 1 bytes per text.
 *   - HC_EHIP reports a failed HIP runtime call or a device that is not
 *     gfx950; HC_ENOMEM a failed allocation.
 */
#ifndef HC_H
#define HC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HC_OK = 0,
    HC_EINVAL = -1,     /* invalid argument; nothing was written            */
    HC_ENOMEM = -2,     /* host or device allocation failed                  */
    HC_EOVERFLOW = -3,  /* more results than `cap`; the true total is
                           reported and the first `cap` results are written  */
    HC_EAGAIN = -4,     /* served request not finished yet                   */
    HC_EHIP = -5        /* HIP runtime error, or no gfx950 device            */
} hc_status;

/*
 * Method parameters (Section 3.2; Section 4 explores 1 <= q <= 8 and
 * 8 <= alpha <= 12). A field set to 0 is chosen by the library.
 *   q      q-gram length, 1 <= q <= min(m, 8).
 *   alpha  F has 2^alpha words (the hash h is reduced mod 2^alpha, eq. (3)).
 *   w      bits per word of F, one of 8, 16, 32, 64 (the link hash of eq. (5)
 *          maps a hash v to bit v mod w). Limits: 1 <= alpha and
 *          2^alpha * w / 8 <= 64 KiB.
 */
typedef struct {
    int32_t q;
    int32_t alpha;
    int32_t w;
} hc_params;

/* Work split inside the search kernel (no effect on results).
 *   segment   each lane runs the search loop over its own block of window
 *             starts (any split of the starts is exact, because every shift
 *             only skips windows that cannot match, Section 3.3);
 *   wave      the 64 lanes of a wavefront try 64 consecutive windows and the
 *             wavefront moves on to the furthest position any lane proved
 *             safe (shift agreement across the wavefront);
 *   dense     every window of the text gets the test the search loop applies
 *             (first word, then the chain of links back to the window start,
 *             then H_v), no shifts; the surviving windows are verified. For
 *             short shifts (m - q + 1 small), where the loop saves little,
 *             this avoids its divergence. Available for patterns without
 *             links (m < 2q, any q) and for q <= 4 with up to 3 links per
 *             window; other patterns run the segment schedule. With
 *             4 <= m <= 8 and no links the window (one or two dwords) is
 *             compared with x directly, which decides exactly what test
 *             plus verification decide. */
enum { HC_SCHED_AUTO = 0, HC_SCHED_SEGMENT = 1, HC_SCHED_WAVE = 2, HC_SCHED_DENSE = 3 };

/* Searching-phase variant (no effect on results).
 *   hc        the plain searching phase (Section 3.3);
 *   sentinel  SHC (Section 3.4, third optimisation): a copy of x is placed
 *             after each text tile in on-chip memory, so the loop over
 *             empty words runs without a position test (a lane's loop may
 *             run into the next lane's range before it stops). Kept for
 *             reference and parity only: with many lanes per tile the
 *             overrun costs far more than the saved test, so it is slower
 *             than `hc` everywhere and the library never chooses it;
 *   sparse    for long patterns: no tile is staged; each lane reads the
 *             q-grams it hashes (and the windows it verifies) in place, so
 *             only the cache lines that hold them are fetched; long chain
 *             walks and verifications are shared by a whole wavefront.
 *             Tiles hold 256 * segment window starts (segment 0 = 1024, up
 *             to 4096), the segment rounded to a whole number of shifts
 *             (m - q + 1) when the shift is 32..4096 starts; one tile per
 *             workgroup unless wg_per_cu caps the grid.
 * The sentinel variant ignores the schedule (one range per lane). */
enum { HC_VARIANT_AUTO = 0, HC_VARIANT_HC = 1, HC_VARIANT_SENTINEL = 2, HC_VARIANT_SPARSE = 3 };

/* Launch shape of the search kernel. A field set to 0 is chosen by the
 * library (the autotuner's cache, else built-in priors: the dense schedule
 * on tiles of 16384 starts for patterns without links, m < 2q, which the
 * default q gives every m <= 8;
 * else the segment schedule on tiles of 25600 starts). */
typedef struct {
    int32_t segment;     /* window starts per lane; tile = 256 * segment     */
    int32_t schedule;    /* HC_SCHED_*                                        */
    int32_t variant;     /* HC_VARIANT_*                                      */
    int32_t wg_per_cu;   /* resident workgroups per compute unit, 1..8        */
} hc_launch;

typedef struct hc_pattern hc_pattern;   /* opaque; immutable once built      */

/*
 * hc_autotune -- measure the fastest parameters for each pattern length in
 * ms[0..n_ms) on the device text d_y[0..n) (n <= 4 GiB, 1 <= m <= min(n,
 * 4096)), and make them the library's choice for fields left at 0 (hc_params
 * of hc_preprocess and batch plans, segment and schedule of hc_launch) for
 * every pattern whose length falls in the same bucket (2^(b-1), 2^b]; the
 * last tuning of a bucket wins, process-wide. Candidates: q in [1, min(m,
 * 8)], (alpha, w) in {(8,8), (10,16), (11,16), (12,16), (12,32)}, the segment
 * and dense schedules, segments {48, 64, 80, 100}, and for m >= 256 the
 * sparse variant with segments of 1, 2, 4 or 8 shifts (m - q + 1, at most
 * 4096 starts); timed with `patterns`
 * (1..64) patterns copied from the text at fixed pseudo-random offsets.
 * out[i] (may be NULL) receives the choice for ms[i] and its median text
 * GB/s. Runs on `stream` and synchronises it; allocates a scratch output of
 * min(n, 2^25) positions and, when it fits, a 512 MiB buffer that is
 * overwritten before each timed launch (so the text is read from HBM, not
 * from the last-level cache). The choice never changes search results (the
 * parameters only change speed). Errors: HC_EINVAL on bad arguments.
 * hc_autotune_reset forgets every tuned entry.
 */
typedef struct {
    int64_t m;
    hc_params params;
    hc_launch launch;
    double gbps;
} hc_tuning;

hc_status hc_autotune(const uint8_t *d_y, int64_t n, const int64_t *ms, int32_t n_ms,
                      int32_t patterns, hc_tuning *out, void *stream);
void hc_autotune_reset(void);

/*
 * hc_preprocess -- the preprocessing phase (Section 3.1, eqs. (1)-(2);
 * Section 3.4 first and second optimisations): builds the word vector F,
 * the shift s = floor(alpha/q) (eq. (4)), the mask F' = 2^alpha - 1 and the
 * chain-head hash H_v for pattern x[0..m-1] (host bytes, copied).
 *   params  may be NULL (all fields chosen by the library).
 *   *out    receives a pattern object owned by the caller, released with
 *           hc_pattern_free(). It may be shared by threads and streams.
 * Errors: m < 1 or m > 4096, q outside [1, min(m, 8)], w not in
 * {8,16,32,64}, alpha outside [1, alpha_max(w)] -> HC_EINVAL.
 * Host-only: no device is touched until the first search.
 */
hc_status hc_preprocess(const uint8_t *x, int64_t m, const hc_params *params,
                        hc_pattern **out);

/*
 * hc_pattern_info -- read back what hc_preprocess built (for F-table parity
 * checks). Any output pointer may be NULL. *F_host points at 2^alpha words
 * stored as uint64_t (low w bits used), valid while the pattern lives;
 * *F_words = 2^alpha.
 */
hc_status hc_pattern_info(const hc_pattern *p, hc_params *used, int32_t *s,
                          uint32_t *mask, uint32_t *hv, const uint64_t **F_host,
                          int64_t *F_words, int64_t *m);

void hc_pattern_free(hc_pattern *p);

/*
 * hc_preprocess_many -- the preprocessing phase (as hc_preprocess) for n
 * patterns at once, computed on the device: one workgroup per pattern sets
 * the links of eq. (1) with atomic ORs in on-chip memory, then, after a
 * barrier, the first-q marks of eq. (2) into words still empty (Section 3.4),
 * and writes F as 2^alpha packed w-bit words (little-endian, the layout of
 * hc_pattern_info's words truncated to w bits) at d_F + i * table_stride.
 *   pat/pat_off  (host) pattern bytes and n + 1 offsets; 1 <= m <= 4096;
 *   params       alpha and w shared by all patterns (0 = 12 and 32); q per
 *                pattern (0 = library choice, capped at m);
 *   d_F          device memory of n * table_stride bytes (caller-owned);
 *   table_stride a multiple of 16, >= max(16, 2^alpha * w / 8), at most the
 *                on-chip memory of one workgroup (160 KiB);
 *   used, info   (host, may be NULL) per pattern: the parameters used, and
 *                s, mask, H_v (three uint32 each).
 * Synchronises `stream`. The tables equal hc_preprocess's bit for bit.
 */
hc_status hc_preprocess_many(const uint8_t *pat, const int64_t *pat_off, int32_t n,
                             const hc_params *params, void *d_F, int64_t table_stride,
                             hc_params *used, uint32_t *info, void *stream);

/*
 * hc_search -- the searching phase (Section 3.3): all occurrences of the
 * pattern in d_y[0..n-1] (device bytes).
 *   d_out   device int64 array of `cap` entries; receives the first
 *           min(count, cap) occurrences, ascending.
 *   *count  (host) the true number of occurrences.
 * Synchronises `stream` to read the count. count > cap -> HC_EOVERFLOW with
 * the first `cap` results written. n < m -> HC_OK, count 0.
 */
hc_status hc_search(const hc_pattern *p, const uint8_t *d_y, int64_t n,
                    int64_t *d_out, int64_t cap, int64_t *count, void *stream);

/*
 * hc_search_async -- as hc_search, without a host synchronisation: the total
 * is written to *d_count (device int64) in stream order, and positions past
 * `cap` are dropped without an error (compare *d_count with cap afterwards).
 *   launch  may be NULL (library choice).
 * The total is written by the second of the call's two kernels (the one
 * that writes the ordered positions), after all tiles were searched.
 */
hc_status hc_search_async(const hc_pattern *p, const uint8_t *d_y, int64_t n,
                          int64_t *d_out, int64_t cap, int64_t *d_count,
                          const hc_launch *launch, void *stream);

/*
 * hc_search_async_noalloc -- hc_search_async for callers that cannot
 * allocate device memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation). Same arguments,
 * results and stream ordering as hc_search_async, and the same two kernels;
 * the per-tile results between them go to a fixed 64 MiB device array that
 * the library holds on each device it runs on (until the process ends)
 * instead of the per-stream workspace. The call allocates nothing:
 *   - the pattern must already have its device copy on the current device
 *     (made by any earlier hc_search / hc_search_async with it there), else
 *     HC_EINVAL;
 *   - a call whose per-tile results need more than 64 MiB gives HC_EINVAL
 *     (they take 4 + 512 + tile/8 bytes per tile of `tile` window starts:
 *     texts up to about 420 MiB at the default tile shapes);
 *   - the first call on a device looks up the array's address and, like any
 *     first launch of a kernel shape, fills host-side caches.
 * Every call on one device shares the array: calls that overlap on that
 * device (on different streams or from different threads without ordering)
 * race and give wrong results; calls ordered on one stream are safe. Nothing
 * in the array needs clearing between calls.
 */
hc_status hc_search_async_noalloc(const hc_pattern *p, const uint8_t *d_y, int64_t n,
                                  int64_t *d_out, int64_t cap, int64_t *d_count,
                                  const hc_launch *launch, void *stream);

/*
 * Batched search: every listed (pattern, text) pair in one persistent launch
 * (one text tile is staged on chip once and searched for many patterns).
 *   d_text            device bytes holding all texts;
 *   text_off[k]       (host) byte offset of text k in d_text, n_texts + 1
 *                     entries, non-decreasing;
 *   pat / pat_off     (host) all pattern bytes and n_pats + 1 offsets;
 *   pair_pat/pair_text (host) pattern and text index of each of n_pairs pairs.
 * Result (CSR, device): the occurrences of pair k are
 * d_pos[d_pair_off[k] .. d_pair_off[k+1]) ascending; d_pair_off has
 * n_pairs + 1 entries. *total (host) = all occurrences. total > cap ->
 * HC_EOVERFLOW; then d_pair_off still holds the full offsets but d_pos holds
 * only positions whose slot is < cap. Synchronises `stream`. Positions are
 * gathered in a device scratch buffer first (grown when a run needs more,
 * then the run is repeated once); a batch that would need 2^32 - 1 or more
 * scratch positions gives HC_ENOMEM (split it).
 *   params  NULL = q chosen per pattern (autotuner / priors), alpha = 12, w = 16.
 */
typedef struct {
    const uint8_t *d_text;
    const int64_t *text_off;
    int32_t n_texts;
    const uint8_t *pat;
    const int64_t *pat_off;
    int32_t n_pats;
    const int32_t *pair_pat;
    const int32_t *pair_text;
    int64_t n_pairs;
} hc_batch;

hc_status hc_search_batched(const hc_batch *batch, const hc_params *params,
                            int64_t *d_pos, int64_t cap, int64_t *d_pair_off,
                            int64_t *total, void *stream);

/*
 * Batch plans: hc_search_batched split in two, for batches searched many
 * times. hc_batch_plan_create preprocesses every pattern (the word vectors of
 * one batch share alpha and w; w must be 16 or 32 and 2^alpha * w / 8 at most
 * 16 KiB, else HC_EINVAL; params->q, when set,
 * applies to every pattern, capped at its length), groups the pairs by text
 * and uploads the work list. The texts stay caller-owned and must outlive the
 * plan. hc_batch_plan_run searches (results and errors as hc_search_batched)
 * by replaying a HIP graph captured for its (d_pos, cap, d_pair_off, stream);
 * runs of one plan must not overlap. hc_batch_plan_free releases the plan.
 */
typedef struct hc_batch_plan hc_batch_plan;

hc_status hc_batch_plan_create(const hc_batch *batch, const hc_params *params,
                               hc_batch_plan **out);
hc_status hc_batch_plan_run(hc_batch_plan *plan, int64_t *d_pos, int64_t cap,
                            int64_t *d_pair_off, int64_t *total, void *stream);
void hc_batch_plan_free(hc_batch_plan *plan);

/*
 * hc_batch_autotune -- measure which table shape (alpha, w), lane segment,
 * patterns per staged tile (group) and resident workgroups per compute unit
 * make batch plans fastest on this batch (on an evenly spaced sample of at
 * most max_pairs of its pairs), and make them the library's choice for batch
 * plans, hc_search_batched and servers created afterwards with params NULL
 * (or alpha and w left at 0); process-wide, the last tuning wins, and
 * hc_autotune_reset forgets it. q stays per pattern (hc_autotune's tuning or
 * the built-in priors). out (may be NULL) receives the choice and its
 * pattern x text GB/s on the sample. Builds and runs several plans on
 * `stream` and synchronises it; allocates their outputs. The choice never
 * changes results. Errors: HC_EINVAL on bad arguments or an empty batch.
 */
typedef struct {
    hc_params params;     /* alpha and w chosen (q = 0: per pattern)          */
    int32_t segment;      /* window starts per lane of the batched kernel      */
    int32_t group;        /* patterns searched per staged tile                 */
    int32_t wg_per_cu;    /* cap on resident workgroups per CU (0 = none)      */
    double gbps;          /* pattern x text bytes per second on the sample     */
} hc_batch_tuning;

hc_status hc_batch_autotune(const hc_batch *batch, int64_t max_pairs, hc_batch_tuning *out,
                            void *stream);

/*
 * Serving: continuous batching of search requests against resident texts.
 * hc_serve_create registers n_texts device texts (caller-owned, written
 * before the call, must outlive the server), a device-memory budget in bytes
 * for in-flight requests, and optional params shared by every request (as
 * for batch plans: NULL = q per pattern, alpha 12, w 16; w 16 or 32, tables
 * up to 16 KiB). Each in-flight request holds its table, a 4128-byte pattern
 * slot and room for 4096 positions per step (32 KiB); a budget below one
 * request's share gives HC_EINVAL. A scheduler thread admits queued requests
 * (FIFO) while the budget allows, and runs steps: one batched launch searches
 * the next 64 MiB chunk of every text that has active requests, for all of
 * them. A request that arrives while others run joins at the next step and
 * finishes after one full cycle over its text. Results are the same as
 * hc_search's, whatever else is in flight.
 * hc_serve_submit preprocesses and copies x (1 <= m <= 4096) and returns a
 * request id (thread-safe).
 * hc_serve_poll waits up to timeout_us (0 = do not wait) and returns
 * HC_EAGAIN while the request runs; when done it copies min(count, cap)
 * ascending positions to host `out` and sets *count. With count <= cap it
 * releases the request and returns HC_OK; otherwise it returns HC_EOVERFLOW
 * and keeps the request, so a second poll with cap >= count gets all of it.
 * An unknown or released id gives HC_EINVAL; a failed step fails its requests
 * with that step's status (HC_EHIP, HC_ENOMEM) and later submits with it too.
 * Stats: latency percentiles of completed requests (submit to completion),
 * aggregate text bytes searched (summed over requests) per second of time the
 * scheduler spent in steps, and the number of completed requests.
 */
typedef struct hc_server hc_server;

hc_status hc_serve_create(const uint8_t *const *d_texts, const int64_t *n,
                          int32_t n_texts, int64_t device_mem_budget,
                          const hc_params *params, hc_server **out);
hc_status hc_serve_submit(hc_server *s, int32_t text_id, const uint8_t *x,
                          int64_t m, uint64_t *req_id);
hc_status hc_serve_poll(hc_server *s, uint64_t req_id, int64_t *out, int64_t cap,
                        int64_t *count, int32_t timeout_us);
/* hc_serve_next_done waits up to timeout_us for a completed request that
 * has not been reported yet and not been released, and returns its id (each
 * id once, in completion order); HC_EAGAIN when none completed in time. */
hc_status hc_serve_next_done(hc_server *s, uint64_t *req_id, int32_t timeout_us);
hc_status hc_serve_stats(hc_server *s, double *p50_us, double *p99_us,
                         double *agg_gbps, int64_t *done);
hc_status hc_serve_destroy(hc_server *s);

const char *hc_strerror(hc_status st);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */
