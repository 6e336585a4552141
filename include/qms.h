/*
 * qms.h -- QuickMergesort on AMD Instinct MI355X (gfx950): the C ABI of
 * libqms.so.
 *
 * The method (Edelkamp & Weiss, "QuickMergesort: Practically Efficient
 * Constant-Factor Optimal Sorting", Sec. "QuickXsort and QuickMergesort",
 * Fig. 2): a median-of-3 pivot partitions the array; the smaller side is
 * sorted by Mergesort while the other side serves as swap space (every
 * element Mergesort would move out is exchanged with a buffer element); the
 * loop continues on the larger side.  Each array is sorted in place.
 *
 * Conventions shared by every entry point:
 *   - Key and payload buffers are DEVICE memory owned by the caller (for
 *     example allocated by torch).  They are sorted in place; the library
 *     never frees or reallocates them.  Pointers must be 4-byte aligned.
 *   - Keys are 32-bit words: QMS_U32 compares them as unsigned integers;
 *     QMS_F32 compares IEEE-754 binary32 values by the IEEE total order
 *     (negative NaNs < -inf < ... < -0 < +0 < ... < +inf < positive NaNs).
 *     Every sorting entry point also takes 64-bit keys (the wide records of
 *     the paper's Experiments section): QMS_U64 unsigned, QMS_F64 IEEE-754
 *     binary64 by the same total order; 8-byte aligned, with or without
 *     payloads (with payloads their merge passes are 2-way and their base
 *     tile is 2048 keys).
 *   - QMS_U32_LOG: uint32 keys under an expensive comparison, the
 *     logarithm of each key in double precision evaluated inside every
 *     comparison (the comparator of the paper's Experiments section that
 *     makes element comparisons costly).  log is strictly increasing and
 *     double precision separates the logarithms of distinct keys below
 *     2^32, so the result is the QMS_U32 sort; what changes is the cost of
 *     each comparison in the partition, the merges and the base case.  Keys
 *     only (QMS_ERR_UNSUPPORTED with payloads).
 *   - Payloads (qms_sort_pairs, qms_sort_batch with vals) are uint32 words in
 *     a separate array (structure of arrays); every move of a key moves its
 *     payload.  The sort is not stable: payload order among equal keys is
 *     unspecified, as both the partition and the merge reorder equal keys.
 *   - `stream` is a hipStream_t (0 = the null stream).  Work is enqueued on
 *     that stream.  The single-array entry points read small partition
 *     results back to the host once per partition round, so they return
 *     only after the sort has completed on the stream.
 *   - Extra device memory: a library-owned workspace per (device, stream)
 *     of fixed size, about 370 MB (tile counters, run samples, split
 *     vectors, task tables and the round state of device-planned batches;
 *     nothing proportional to n), allocated on first use and kept until
 *     qms_release_workspaces().  Every sort is in place: no key or payload
 *     is ever held outside the caller's arrays.
 *   - Return values are qms_status codes; no C++ exception crosses this
 *     interface.  The message of the last failure on the calling thread is
 *     available from qms_last_error().
 *   - Threads: every entry point may be called from any host thread.  Sorts
 *     issued on the same (device, stream) share that stream's workspace and
 *     run one after another (a call waits for another thread's call on the
 *     same stream to return); sorts on different streams run concurrently.
 */
#ifndef QMS_H
#define QMS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMS_U32 = 0,
    QMS_F32 = 1,
    QMS_U64 = 2,
    QMS_F64 = 3,
    QMS_U32_LOG = 4 /* uint32 keys compared by log(key) (see above) */
} qms_dtype;

typedef enum {
    QMS_OK = 0,
    QMS_PENDING = 1,         /* server: request not finished yet          */
    QMS_ERR_INVALID = -1,    /* bad argument (NULL, host pointer, range)  */
    QMS_ERR_ALIGN = -2,      /* pointer not 4-byte aligned                */
    QMS_ERR_NOMEM = -3,      /* workspace allocation failed               */
    QMS_ERR_HIP = -4,        /* a HIP runtime call or kernel failed       */
    QMS_ERR_BUDGET = -5,     /* server: request larger than the budget    */
    QMS_ERR_UNSUPPORTED = -6 /* unknown dtype or option                   */
} qms_status;

/*
 * qms_sort -- sort n keys in place (Fig. 2 sort(); Sec. "QuickXsort and
 * QuickMergesort"; pivot rule of Theorem 1: median of the keys at lo,
 * lo + (hi-lo)/2 and hi-1).
 *   d_keys  device pointer to n keys of type dt (4 or 8 bytes each).
 *   n       number of keys; 0 and 1 are no-ops returning QMS_OK.  At most
 *           2^32 + 2^25: a round whose range holds 2^32 keys or more
 *           partitions it as blocks of 2^31 keys around the pivot of the
 *           whole range and gathers the blocks' classes by in-place
 *           rotations; the bound keeps every Mergesort side (at most half
 *           a range) within the workspace's merge tables.
 *   dt      QMS_U32, QMS_F32, QMS_U64, QMS_F64 or QMS_U32_LOG.
 *   stream  HIP stream to run on.  When `stream` is being captured into a
 *           HIP graph, the call reads nothing back: its rounds are planned
 *           on the device, as qms_sort_batch plans a batch of one array
 *           (n below 2^32; the range left at final_tile keys or below is
 *           sorted by the bitonic network, as without capture), and it
 *           returns at once.  A first call on the stream outside the
 *           capture allocates the stream's workspace.
 * Errors: QMS_ERR_INVALID for NULL with n > 0 or a pointer that is not
 * device memory; QMS_ERR_ALIGN; QMS_ERR_UNSUPPORTED for an unknown dt or
 * n above the bound; QMS_ERR_NOMEM / QMS_ERR_HIP from the runtime.
 */
int qms_sort(void *d_keys, uint64_t n, int dt, hipStream_t stream);

/*
 * qms_sort_pairs -- as qms_sort, carrying a uint32 payload per key (the
 * QuickXsort section's element moves apply to whole elements).
 *   d_vals  device pointer to n uint32 payloads, permuted with the keys.
 *   dt      any key type (QMS_U32, QMS_F32, QMS_U64, QMS_F64).
 * Result: keys sorted; the multiset of (key, payload) pairs preserved.
 */
int qms_sort_pairs(void *d_keys, uint32_t *d_vals, uint64_t n, int dt,
                   hipStream_t stream);

/*
 * qms_sort_batch -- sort num_segments independent arrays stored back to back
 * (segment j is [offsets[j], offsets[j+1])), each exactly as qms_sort /
 * qms_sort_pairs would, with all segments advancing together through the
 * partition / base-case / merge phases (one set of launches per phase for
 * the whole batch rather than per segment).  The rounds are planned on the
 * device: the call enqueues a fixed schedule of launches on `stream` and
 * returns without waiting for the GPU (no readback, no synchronisation),
 * so it may be captured into a HIP graph (after one call outside the
 * capture, which allocates the stream's workspace).  The schedule: a
 * number of rounds that follows from the longest segment (1.2 rounds per
 * binary level above the base tile, plus two), with the paper's pivot rule
 * (median-of-3, after an unbalanced round the median of the medians of
 * three: Sec. "Worst-Case Efficient QuickMergeSort"); then every range still
 * above the base tile is sorted in place by a bitonic network (X at the
 * loop level, as the single-array loop finishes its last range), so every
 * segment is sorted whatever its keys.  final_tile is not used: the loop
 * runs down to the base tile while the rounds last.
 *   d_keys       device keys of all segments.
 *   d_vals       device uint32 payloads (one per key), or NULL for keys
 *                only.
 *   d_offsets    DEVICE array of num_segments + 1 uint64 offsets, non-
 *                decreasing, offsets[0] = 0 (empty segments allowed).
 *   h_offsets    HOST copy of the same offsets; NULL makes the library read
 *                them from the device first (a synchronisation of `stream`).
 * Errors: as qms_sort; QMS_ERR_INVALID for decreasing offsets;
 * QMS_ERR_UNSUPPORTED for a segment of 2^32 keys or more.
 */
int qms_sort_batch(void *d_keys, uint32_t *d_vals, const uint64_t *d_offsets,
                   const uint64_t *h_offsets, uint32_t num_segments, int dt,
                   hipStream_t stream);

/*
 * qms_batch_check -- wait for `stream` (current device) and report whether
 * every qms_sort_batch enqueued on it since the last check finished within
 * its schedule: QMS_OK, or QMS_ERR_HIP with the number of segments left
 * unsorted in qms_last_error() (the schedule's bound makes this a check of
 * the library itself; it has no other cause).  Resets the count.
 */
int qms_batch_check(hipStream_t stream);

/*
 * qms_sort_noalloc -- qms_sort for callers that cannot allocate memory: code
 * under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and errors as qms_sort, for at most
 * 2^28 keys (QMS_ERR_UNSUPPORTED above that).  It allocates nothing: no
 * hipMalloc or hipFree, no pinned host memory, no events.  The kernels' tile
 * counters, split vectors and run samples live in a fixed 32 MiB device
 * array of the library (one per GPU, held until the process ends) instead
 * of a cached workspace (the last ranges are finished in place, as by
 * qms_sort, so no other buffer is needed).  Calls on one GPU share that
 * array: calls are
 * serialised on the host, but calls whose GPU work overlaps (other streams
 * of the same device, not synchronised between the calls) race on it.  Like
 * qms_sort it reads partition results back once per round.
 */
int qms_sort_noalloc(void *d_keys, uint64_t n, int dt, hipStream_t stream);

/* ---- request loop (serving) ---------------------------------------------
 * A server owns a worker thread and a HIP stream on `device`.  Requests are
 * device arrays lent to the server until qms_server_poll returns QMS_OK for
 * their ticket.  Admission: the bytes of all lent, unfinished requests stay
 * within hbm_budget_bytes; requests beyond it wait in FIFO order (none is
 * dropped).  Pending requests are grouped by dtype into batches of at most
 * max_batch requests and sorted with the batched path.
 */
typedef struct {
    uint64_t hbm_budget_bytes; /* admission budget for lent key+payload bytes */
    int device;                /* HIP device ordinal                          */
    uint32_t max_batch;        /* max requests per batch (0: 4096)            */
} qms_server_config;

typedef struct qms_server qms_server;

/* Create a server.  *out receives the handle. */
int qms_server_create(const qms_server_config *cfg, qms_server **out);

/*
 * Submit one request: sort n keys of dtype dt (any qms_dtype; 8-byte aligned
 * for 64-bit keys) at d_keys (device memory of the server's device), in
 * place.  `stream` is the stream whose work produced the keys: the server
 * records an event on it at submit and sorts the request only after the
 * work enqueued there before the submit has run (0 = the null stream).
 * *ticket_out receives a ticket.  Returns QMS_ERR_BUDGET if the request's
 * n * 4 (64-bit keys: n * 8) bytes alone exceed the budget (never
 * admissible), QMS_ERR_UNSUPPORTED for an unknown dtype, QMS_ERR_HIP if the
 * event cannot be recorded on `stream`.
 */
int qms_server_submit(qms_server *srv, void *d_keys, uint64_t n, int dt,
                      hipStream_t stream, uint64_t *ticket_out);

/*
 * Poll a ticket: QMS_PENDING while queued or running; QMS_OK once the keys
 * are sorted (the ticket is then retired and *latency_s_out, if not NULL,
 * receives completion time minus submission time in seconds);
 * QMS_ERR_INVALID for an unknown or retired ticket; QMS_ERR_HIP if the
 * batch holding the request failed.
 */
int qms_server_poll(qms_server *srv, uint64_t ticket, double *latency_s_out);

/* Statistics since creation: completed requests, completed keys, peak
 * admitted bytes, and requests that had to wait for budget. */
typedef struct {
    uint64_t completed;
    uint64_t completed_keys;
    uint64_t peak_admitted_bytes;
    uint64_t waited_for_budget;
    uint64_t batches;
} qms_server_stats;
int qms_server_get_stats(qms_server *srv, qms_server_stats *out);

/* Drain in-flight work, stop the worker and free the server. */
int qms_server_destroy(qms_server *srv);

/* ---- diagnostics ---------------------------------------------------------- */

/* Message of the last failure on the calling thread ("" if none). */
const char *qms_last_error(void);

/* Free the cached workspaces of all devices and streams.  A workspace in use
 * (a sort running on another thread, or a live server's) is kept, and
 * QMS_ERR_INVALID reports that one was. */
int qms_release_workspaces(void);

/*
 * Round log of the last single-array sort on the calling thread: for each
 * partition round, the range size s, the sizes of the sides (<, ==, >
 * pivot; == is 0 when the few pivot-equal keys stayed with the > side), the
 * number of merge levels run on the mergesorted side, and the pivot rule of
 * the round (0 median-of-3, 1 median of the medians of three, taken after a
 * round whose smaller side held less than 1/16 of its range: Sec.
 * "Worst-Case Efficient QuickMergeSort", HybridQuickMergesort with
 * delta = 1/16).  Writes up to max_rounds records of QMS_SCHEDULE_WORDS
 * uint64 each into out; returns the number of rounds of that sort (which
 * may exceed max_rounds).
 */
#define QMS_SCHEDULE_WORDS 6
uint64_t qms_last_schedule(uint64_t *out, uint64_t max_rounds);

/*
 * The worst-case pivot of Sec. "Worst-Case Efficient QuickMergeSort"
 * (MoMQuickMergesort): the lower median of the floor(n/3) medians of the
 * triples (d_keys[3i], d_keys[3i+1], d_keys[3i+2]), keys compared as in
 * qms_sort (dt).  At least 2 floor(n/6) keys are <= it and as many >= it.
 * The same kernels pick the pivot inside a sort after an unbalanced round;
 * this entry point runs them on a whole array, for tests and callers that
 * want the pivot alone.  d_keys: n keys of dtype dt on the current device
 * (read only; 8-byte aligned for 64-bit keys); pivot_out (host) gets the
 * pivot's bits: 4 bytes for QMS_U32, QMS_F32 and QMS_U32_LOG (whose order
 * is the integers' order), 8 bytes for QMS_U64 and QMS_F64.  Synchronises
 * `stream`.  Errors: QMS_ERR_INVALID for NULL pointers or n < 3,
 * QMS_ERR_ALIGN for misaligned keys, QMS_ERR_UNSUPPORTED for n >= 2^32 or
 * an unknown dt, QMS_ERR_HIP.
 */
int qms_mom_pivot(const void *d_keys, uint64_t n, int dt, void *pivot_out,
                  hipStream_t stream);

/*
 * Per-kernel-class timing of the sorts issued by the calling thread between
 * qms_profile_begin and qms_profile_end.  Each launch is bracketed by HIP
 * events recorded on its own stream; qms_profile_end waits for them and
 * returns, per class ("tile_sort", "merge_split", "merge", "part_count",
 * "part_scan", "part_split", "part_swap"), the number of launches, their
 * summed duration and their summed algorithmic bytes (the bytes the method
 * must move: 16 per key per swap-merge level and per swapping base-case
 * pass, 8 per key for an in-place base-case pass, 4 per key for counting,
 * doubled for key/payload pairs), followed by one record per binary level
 * at which swap-merge passes started ("merge_level_<l>"; a 4-way pass covers
 * levels l and l + 1).  Writes up to max_entries records; *n_out gets the
 * number written.
 */
typedef struct {
    char name[32];
    uint64_t launches;
    double total_ms;
    double bytes;
} qms_kernel_stat;
int qms_profile_begin(void);
int qms_profile_end(qms_kernel_stat *out, int max_entries, int *n_out);

/*
 * Run-time tunables, process-wide, read at the start of every sort (the
 * server's worker included); defaults {4, 4096, 16384, 0, 2^22}.  They
 * change speed, never results.
 *   merge_ways      2 or 4: every sort merges four runs per pass (the
 *                   multi-way merging proposed in the paper's Conclusion) or
 *                   two.
 *   partition_tile  keys per counting tile of the partition (a power of two
 *                   in [4096, 65536]); a round with more than 2^20 tiles
 *                   doubles it.
 *   chunk_span      target positions per exchange chunk of the partition, in
 *                   [4096, 2^20] (smaller: more, shorter chunks).
 *   base_tile       X_THRESH of QuickMergeXsort (Sec. "QuickMergeXsort"): the
 *                   Mergesort of each round stops at runs of this many keys,
 *                   which the base case X (a bitonic network in LDS) sorts;
 *                   a power of two in [2048, 16384].  Smaller: fewer network
 *                   comparisons, more merge levels.  Key/payload sorts and
 *                   64-bit keys use at most 8192.  16384 = sqrt(2^28), the
 *                   paper's sqrt(n) rule for the 2^28-key workload.  0
 *                   (automatic): 16384 (8192 for pairs), except that a sort
 *                   merging four runs per pass takes half of that for a
 *                   Mergesort whose level count would otherwise be odd;
 *                   2048 for 64-bit keys, whose network costs more per
 *                   level than a merge level, and for QMS_U32_LOG, whose
 *                   network comparisons cost more than the merges'.
 *   final_tile      a range that a partition round leaves with at most this
 *                   many keys leaves the QuickMergesort loop and is sorted
 *                   in place by X = a bitonic network (QuickXsort with X at
 *                   the loop level; the paper's loop continues to the base
 *                   tile): tiles by the base case, then the network's
 *                   stages above the tile, every exchange between two cells
 *                   of the range.  It adds O(F log^2 F) comparisons for a
 *                   range of F keys.  Every input array above the base tile
 *                   is partitioned at least once; arrays of at most the
 *                   base tile are sorted in place by the base case.  0
 *                   (automatic, the default): 2^24 keys for 32-bit keys,
 *                   2^23 for QMS_U64 and QMS_F64, 2^22 for QMS_U32_LOG,
 *                   whose network comparisons cost the most time (the
 *                   sizes measured fastest for each type); when one loop
 *                   sorts several arrays (a batch of the server), the
 *                   smallest power of two p >= the base tile for which
 *                   (arrays longer than p) * p reaches four times that
 *                   size, if there is one below it; else a power
 *                   of two in [8192, 2^30]; 8192 keeps
 *                   every range in the loop down to the base tile, as in
 *                   the paper.  Used by the host-planned loop (qms_sort,
 *                   qms_sort_pairs, qms_sort_noalloc, the server) and by
 *                   qms_sort under capture; qms_sort_batch loops down to
 *                   the base tile.
 * qms_set_tuning returns QMS_ERR_INVALID for values out of range (nothing is
 * changed then).  The package's autotuner (paper_1804_10062_amd/autotune.py)
 * picks them for a workload by timing sorts of a sample.
 */
typedef struct {
    uint32_t merge_ways;
    uint32_t partition_tile;
    uint32_t chunk_span;
    uint32_t base_tile;
    uint32_t final_tile;
} qms_tuning;
int qms_set_tuning(const qms_tuning *t);
int qms_get_tuning(qms_tuning *t);

/* Build-time tiles of the kernels: base-case workgroup tile (keys; the
 * largest base_tile), merge tile, partition tile (elements).  Read-only; for
 * reports and tests. */
void qms_get_tiles(uint32_t *base_tile, uint32_t *merge_tile,
                   uint32_t *partition_tile);

#ifdef __cplusplus
}
#endif

#endif /* QMS_H */
