/*
 * qms_oracle.c -- CPU oracle for QuickMergesort with median-of-3 pivots.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark have a plain, sequential, obviously correct
 * statement of what the method computes.  It shares no code, header, table or
 * helper with the HIP implementation.
 *
 * What it follows (Edelkamp & Weiss, "QuickMergesort: Practically Efficient
 * Constant-Factor Optimal Sorting"):
 *   - the QuickXsort scheme: partition, sort one side with X = Mergesort while
 *     the other side serves as swap space, continue on the rest
 *     (Sec. "QuickXsort and QuickMergesort");
 *   - swap-instead-of-move: an element Mergesort would move to extra space is
 *     exchanged with the element occupying that buffer cell (same section);
 *   - the merge / msort / out / sort routines of Fig. 2 (QuickMergeXsort with
 *     X_THRESH = 2, i.e. pure Mergesort), with two repairs of the printed
 *     figure, both listed below;
 *   - median-of-3 pivot ("CleverQuickMergesort", Theorem 1 / Corollary 2):
 *     3 comparisons for the sample, one comparison per remaining element
 *     during partitioning (proof of Theorem 1);
 *   - QuickMergeXsort (Sec. "QuickMergeXsort", Theorem "Average-Case
 *     QuickMergeXsort"): msort hands ranges shorter than X_THRESH to a
 *     sorting algorithm X and then exchanges the sorted block with its target
 *     cells (the joint movement of Fig. 2).  X = CleverQuicksort, Quicksort
 *     with the median-of-3 partition below (Introduction: its average is
 *     (12/7) ln 2 n lg n + O(n) comparisons).  X_THRESH = 2 is QuickMergesort.
 *
 * Readings of the paper taken here (the paper is silent or its figure does
 * not run as printed):
 *   R1  the partition routine is not given in the paper; this oracle uses a
 *       guarded Hoare partition after a median-of-3 compare-exchange of the
 *       first, middle and last elements.  Both scans stop on keys equal to
 *       the pivot, so runs of equal keys split evenly.
 *   R2  the side test of sort() adds two iterators; read as
 *       "b - begin < (end - begin) / 2" with integer division: the smaller
 *       side is sorted by Mergesort, the loop continues on the larger side.
 *   R3  in msort the final merge of the printed figure passes run1 as
 *       [begin+q, begin+n); run1 holds q elements, so for odd n that merge
 *       would consume a buffer element.  Here run1 is [begin+q, begin+2q).
 *   R4  the tail loop of merge reads one cell past endtarget on its last
 *       step; the value read is dead (the hole is closed with temp right
 *       after), so the last step writes temp directly and reads nothing.
 *   R5  ranges of 2 elements are finished with one compare-exchange; ranges
 *       of 0 or 1 element are done (median-of-3 needs 3 elements).
 *   R6  float keys are compared through the IEEE-754 total order (negative
 *       NaNs < -inf < ... < -0 < +0 < ... < +inf < positive NaNs), realised by
 *       flipping the bits of negative values and the sign bit of the others;
 *       with plain '<' the two zeros would tie and the output bits would
 *       depend on the algorithm.
 *   R7  the worst-case pivot of Sec. "Worst-Case Efficient QuickMergeSort"
 *       (qmso_mom_pivot) is the median of n/3 medians of three; the paper
 *       fixes neither the groups nor which middle element of an even count
 *       it means.  Read as the triples (3i, 3i+1, 3i+2), i < floor(n/3), and
 *       the lower median (0-based rank floor((c-1)/2) of the c medians).  The
 *       paper selects it with the median-of-medians algorithm; any exact
 *       selection yields the same value, here a library sort of the medians.
 *   R8  QuickMergeXsort's threshold X_THRESH is one constant for the whole
 *       sort, as in Fig. 2 (msort tests n < X_THRESH); the configuration the
 *       paper analyses, X called at about sqrt(n) elements, takes
 *       X_THRESH = ceil(sqrt(n)) of the whole input (the caller's choice).
 *       CleverQuicksort recurses on the smaller side and loops on the larger
 *       (same comparisons, logarithmic depth) and finishes ranges of two
 *       elements with one compare-exchange (R5).
 *
 * Counters (Experiments section): one comparison per key comparison; one
 * move per element assignment, a swap counting as three moves.  The counting
 * build and the timing build are compiled from this same file
 * (QMSO_COUNTING = 1 / 0), as the paper measured counts and times in
 * separate runs.
 *
 * Elements are (key, payload) when a payload array is given, keys only
 * otherwise; every assignment moves both, every comparison reads keys only.
 *
 * Key width: the file is compiled once with 32-bit keys (entry points
 * qmso_*, qmso_fast_*) and once with 64-bit keys (QMSO_KEY_BITS = 64: the
 * wide records of the Experiments section; qmso64_*, qmso64_fast_*, sort
 * entry points only), the float flag then meaning IEEE-754 binary64 under
 * the same total order (R6).
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef QMSO_COUNTING
#define QMSO_COUNTING 1
#endif

#ifndef QMSO_KEY_BITS
#define QMSO_KEY_BITS 32
#endif

#if QMSO_KEY_BITS == 64
typedef uint64_t qkey_t;
#define KEY_SIGN 0x8000000000000000ull
#if QMSO_COUNTING
#define QMSO_FN(name) qmso64_##name
#else
#define QMSO_FN(name) qmso64_fast_##name
#endif
#else
typedef uint32_t qkey_t;
#define KEY_SIGN 0x80000000u
#if QMSO_COUNTING
#define QMSO_FN(name) qmso_##name
#else
#define QMSO_FN(name) qmso_fast_##name
#endif
#endif

typedef struct {
    uint64_t comparisons;
    uint64_t moves;
} qmso_counters;

/* The array under sort: keys (already in comparable unsigned form),
 * optional payloads, and the counters.  Positions are plain indices. */
typedef struct {
    qkey_t *k;
    uint32_t *v;
    qmso_counters *c;
    size_t xt; /* X_THRESH of msort (2: pure Mergesort) */
} arr_t;

#if QMSO_COUNTING
#define COUNT_CMP(A) ((A)->c->comparisons++)
#define COUNT_MOV(A, x) ((A)->c->moves += (x))
#else
#define COUNT_CMP(A) ((void)0)
#define COUNT_MOV(A, x) ((void)0)
#endif

/* key(i) < key(j), counted as one element comparison */
static inline int less_ij(arr_t *a, size_t i, size_t j)
{
    COUNT_CMP(a);
    return a->k[i] < a->k[j];
}

/* a[dst] := a[src], one move */
static inline void assign(arr_t *a, size_t dst, size_t src)
{
    COUNT_MOV(a, 1);
    a->k[dst] = a->k[src];
    if (a->v) a->v[dst] = a->v[src];
}

/* exchange a[i] and a[j], three moves */
static inline void swap_ij(arr_t *a, size_t i, size_t j)
{
    COUNT_MOV(a, 3);
    qkey_t t = a->k[i];
    a->k[i] = a->k[j];
    a->k[j] = t;
    if (a->v) {
        uint32_t u = a->v[i];
        a->v[i] = a->v[j];
        a->v[j] = u;
    }
}

/*
 * merge (Fig. 2): run1 = [begin1, end1) lies outside the target; run2 lies
 * already in place at [target + (end1 - begin1), endtarget).  The result
 * fills [target, endtarget).  The cells of run1 receive the buffer elements
 * that occupied [target, target + len1) -- the swap principle of the
 * QuickXsort section, done with a travelling hole (temp) so that each merged
 * element costs two moves instead of a three-move swap.  Ties are taken from
 * run2 because the test is the strict key(run1) < key(run2).
 */
static void merge(arr_t *a, size_t begin1, size_t end1, size_t target,
                  size_t endtarget)
{
    size_t i1 = begin1, i2 = target + (end1 - begin1), ires = target;
    qkey_t temp_k = a->k[target];
    uint32_t temp_v = a->v ? a->v[target] : 0;
    COUNT_MOV(a, 1);
    while (i1 != end1 && i2 != endtarget) {
        size_t from = less_ij(a, i1, i2) ? i1++ : i2++;
        assign(a, ires, from); /* chosen element into the hole          */
        ires++;
        assign(a, from, ires); /* next target cell into the vacated cell */
    }
    while (i1 < end1) {
        assign(a, ires, i1);
        ires++;
        if (ires < endtarget) /* R4: the last step reads nothing   */
            assign(a, i1, ires);
        i1++;
    }
    /* close the hole: the buffer element saved at the start */
    a->k[i1 - 1] = temp_k;
    if (a->v) a->v[i1 - 1] = temp_v;
    COUNT_MOV(a, 1);
}

static void clever_quicksort(arr_t *a, size_t lo, size_t hi);

/*
 * msort (Fig. 2): sort [begin, end) into [target, target + n); the buffer
 * elements found at the target end up in [begin, end).  Below X_THRESH the
 * range is sorted by X in place and then swapped into the target cells (the
 * joint movement); with X_THRESH = 2 a single element is its own sorted run.
 */
static void msort(arr_t *a, size_t begin, size_t end, size_t target)
{
    size_t n = end - begin;
    if (n < a->xt) {
        clever_quicksort(a, begin, end);
        for (size_t i = 0; i < n; i++) swap_ij(a, begin + i, target + i);
        return;
    }
    size_t q = n / 2;
    msort(a, begin + q, end, target + q); /* right part into target+q..  */
    msort(a, begin, begin + q, begin + q); /* left part into begin+q..    */
    merge(a, begin + q, begin + 2 * q, target, target + n); /* R3 */
}

/*
 * out (Fig. 2): sort [begin, end) in place, using the ceil(n/2) cells at
 * temp as swap space; those cells get their elements back, permuted.
 */
static void out(arr_t *a, size_t begin, size_t end, size_t temp)
{
    size_t n = end - begin;
    if (n > 1) {
        size_t q = n / 2, r = n - q;
        msort(a, begin + q, end, temp);     /* right r elements -> temp   */
        msort(a, begin, begin + q, begin + r); /* left q -> [begin+r, end) */
        merge(a, temp, temp + r, begin, end);
    }
}

/* compare-exchange so that key(i) <= key(j); one comparison */
static inline void cmp_exchange(arr_t *a, size_t i, size_t j)
{
    if (less_ij(a, j, i)) swap_ij(a, i, j);
}

/*
 * Median-of-3 partition of [lo, hi), hi - lo >= 3 (R1).  Returns b with
 * key[lo..b) <= key[b] <= key(b..hi) and key[b] the pivot.  Exactly
 * hi - lo comparisons: 3 for the sample (lo, lo + s/2, hi - 1) and one for
 * each of the other s - 3 elements (proof of Theorem 1).
 */
static size_t partition(arr_t *a, size_t lo, size_t hi)
{
    size_t s = hi - lo, m = lo + s / 2, l = hi - 1;
    cmp_exchange(a, lo, m);
    cmp_exchange(a, m, l);
    cmp_exchange(a, lo, m); /* key[lo] <= key[m] <= key[l] */
    if (s == 3) return m;
    swap_ij(a, m, lo + 1); /* pivot parked at lo+1          */
    size_t pv = lo + 1;
    size_t i = lo + 2, j = l - 1;
    for (;;) {
        while (i <= j && less_ij(a, i, pv)) i++;
        if (i > j) break;
        while (j > i && less_ij(a, pv, j)) j--;
        if (j == i) break; /* key[i] >= pivot already known */
        swap_ij(a, i, j);
        i++;
        j--;
        if (i > j) break;
    }
    size_t b = i - 1;
    swap_ij(a, pv, b);
    return b;
}

/*
 * X = CleverQuicksort: Quicksort with the median-of-3 partition above on
 * [lo, hi); the smaller side recursively, the larger one by the loop (R8).
 */
static void clever_quicksort(arr_t *a, size_t lo, size_t hi)
{
    while (hi - lo > 1) {
        if (hi - lo == 2) {
            cmp_exchange(a, lo, lo + 1);
            return;
        }
        size_t b = partition(a, lo, hi);
        if (b - lo < hi - (b + 1)) {
            clever_quicksort(a, lo, b);
            lo = b + 1;
        } else {
            clever_quicksort(a, b + 1, hi);
            hi = b;
        }
    }
}

/* sort (Fig. 2): the QuickMergesort loop on [lo, hi). */
static void qms_loop(arr_t *a, size_t lo, size_t hi)
{
    while (hi - lo > 1) {
        if (hi - lo == 2) { /* R5 */
            cmp_exchange(a, lo, lo + 1);
            return;
        }
        size_t b = partition(a, lo, hi);
        if (b - lo < (hi - lo) / 2) { /* R2: left side is the smaller */
            out(a, lo, b, b + 1);
            lo = b + 1;
        } else {
            out(a, b + 1, hi, lo);
            hi = b;
        }
    }
}

/* R6: IEEE-754 total order as an unsigned key, and its inverse (binary32
 * or binary64 by the key width) */
static inline qkey_t f32_bits_to_key(qkey_t u)
{
    return (u & KEY_SIGN) ? ~u : (u | KEY_SIGN);
}
static inline qkey_t key_to_f32_bits(qkey_t k)
{
    return (k & KEY_SIGN) ? (k & ~KEY_SIGN) : ~k;
}

static qmso_counters *counters_or_scratch(qmso_counters *c,
                                          qmso_counters *scratch)
{
    if (c) return c;
    scratch->comparisons = scratch->moves = 0;
    return scratch;
}

/* ---- exported entry points (called from Python through ctypes) ---- */

/* Sort keys (and payloads, if vals != NULL) in place.  is_f32 != 0: the
 * 32-bit words are IEEE-754 binary32 values ordered by R6.  counters may be
 * NULL; otherwise they are accumulated (not reset). */
void QMSO_FN(sort)(qkey_t *keys, uint32_t *vals, size_t n, int is_f32,
                   qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    if (is_f32)
        for (size_t i = 0; i < n; i++) keys[i] = f32_bits_to_key(keys[i]);
    qms_loop(&a, 0, n);
    if (is_f32)
        for (size_t i = 0; i < n; i++) keys[i] = key_to_f32_bits(keys[i]);
}

/* QuickMergeXsort with X = CleverQuicksort below x_thresh (>= 2; R8). */
void QMSO_FN(sort_x)(qkey_t *keys, uint32_t *vals, size_t n, int is_f32,
                     size_t x_thresh, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch),
               x_thresh < 2 ? 2 : x_thresh};
    if (is_f32)
        for (size_t i = 0; i < n; i++) keys[i] = f32_bits_to_key(keys[i]);
    qms_loop(&a, 0, n);
    if (is_f32)
        for (size_t i = 0; i < n; i++) keys[i] = key_to_f32_bits(keys[i]);
}

/* X alone: CleverQuicksort of the whole input. */
void QMSO_FN(clever_quicksort)(qkey_t *keys, uint32_t *vals, size_t n,
                               int is_f32, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    if (is_f32)
        for (size_t i = 0; i < n; i++) keys[i] = f32_bits_to_key(keys[i]);
    clever_quicksort(&a, 0, n);
    if (is_f32)
        for (size_t i = 0; i < n; i++) keys[i] = key_to_f32_bits(keys[i]);
}

/* Sort each segment [offsets[j], offsets[j+1]) independently. */
void QMSO_FN(sort_segments)(qkey_t *keys, uint32_t *vals,
                            const uint64_t *offsets, size_t num_segments,
                            int is_f32, qmso_counters *counters)
{
    for (size_t j = 0; j < num_segments; j++) {
        size_t b = (size_t)offsets[j], e = (size_t)offsets[j + 1];
        QMSO_FN(sort)(keys + b, vals ? vals + b : NULL, e - b, is_f32,
                      counters);
    }
}

#if QMSO_COUNTING && QMSO_KEY_BITS == 32
static int cmp_u32(const void *x, const void *y)
{
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return (a > b) - (a < b);
}

/* R7: the median of the floor(n/3) medians of three (MoMQuickMergesort's
 * pivot, Sec. "Worst-Case Efficient QuickMergeSort"), as the key bits of the
 * input (is_f32: compared by R6).  n >= 3.  Returns 0 and sets *ok = 0 if
 * memory runs out. */
uint32_t qmso_mom_pivot(const uint32_t *keys, size_t n, int is_f32, int *ok)
{
    size_t c = n / 3;
    uint32_t *med = malloc((c ? c : 1) * sizeof(uint32_t));
    *ok = med != NULL && c > 0;
    if (!*ok) {
        free(med);
        return 0;
    }
    for (size_t i = 0; i < c; i++) {
        uint32_t x = keys[3 * i], y = keys[3 * i + 1], z = keys[3 * i + 2];
        if (is_f32) {
            x = f32_bits_to_key(x);
            y = f32_bits_to_key(y);
            z = f32_bits_to_key(z);
        }
        /* median of three: the one that is neither the smallest nor the largest */
        uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
        med[i] = z < lo ? lo : (z > hi ? hi : z);
    }
    qsort(med, c, sizeof(uint32_t), cmp_u32);
    uint32_t p = med[(c - 1) / 2];
    free(med);
    return is_f32 ? key_to_f32_bits(p) : p;
}

/* The pieces below are exported only from the counting build, for tests
 * that pin the individual routines of Fig. 2.  Keys are plain u32. */

size_t qmso_partition(uint32_t *keys, uint32_t *vals, size_t lo, size_t hi,
                      qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    return partition(&a, lo, hi);
}

void qmso_out(uint32_t *keys, uint32_t *vals, size_t begin, size_t end,
              size_t temp, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    out(&a, begin, end, temp);
}

void qmso_msort(uint32_t *keys, uint32_t *vals, size_t begin, size_t end,
                size_t target, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    msort(&a, begin, end, target);
}

/* msort with X = CleverQuicksort below x_thresh (QuickMergeXsort's msort) */
void qmso_msort_x(uint32_t *keys, uint32_t *vals, size_t begin, size_t end,
                  size_t target, size_t x_thresh, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch),
               x_thresh < 2 ? 2 : x_thresh};
    msort(&a, begin, end, target);
}

void qmso_merge(uint32_t *keys, uint32_t *vals, size_t begin1, size_t end1,
                size_t target, size_t endtarget, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    merge(&a, begin1, end1, target, endtarget);
}
#endif
