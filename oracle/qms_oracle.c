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
 *     here every placement is such an exchange (swap_merge, sort_to);
 *   - top-down Mergesort with a buffer: a range is split into its first
 *     floor(n/2) and last ceil(n/2) elements, each half is sorted into the
 *     cells that Fig. 1 shows, and the halves are merged (sort_to,
 *     sort_with_buffer), driven by the QuickMergesort loop of the same
 *     section (quick_merge_sort);
 *   - median-of-3 pivot ("CleverQuickMergesort", Theorem 1 / Corollary 2):
 *     3 comparisons for the sample, one comparison per remaining element
 *     during partitioning (proof of Theorem 1);
 *   - QuickMergeXsort (Sec. "QuickMergeXsort", Theorem "Average-Case
 *     QuickMergeXsort"): the Mergesort hands ranges shorter than X_THRESH to a
 *     sorting algorithm X and then exchanges the sorted block with its target
 *     cells (a joint movement).  X = CleverQuicksort, Quicksort
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
 *   R3  Fig. 2's Mergesort into a target passes its first merged run as n -
 *       floor(n/2) cells long, one more than that run holds for odd n (the
 *       merge would take in a buffer element); here that run is the
 *       floor(n/2) sorted first-half elements.
 *   R4  Fig. 2 realises the exchanges with a travelling hole (two moves per
 *       placed element plus two).  This oracle performs the exchanges of the
 *       swap principle themselves (three moves each): the comparisons, their
 *       outcomes and the sorted result are the same, only the order in which
 *       the buffer elements come back differs, and the move counter reads
 *       three per placed element.
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
 *       sort, as in Fig. 2 (the Mergesort tests n < X_THRESH); the configuration the
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
    size_t xt; /* X_THRESH of the Mergesort (2: pure Mergesort) */
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

/* exchange the k elements at [x, x + k) with those at [y, y + k) */
static void swap_blocks(arr_t *a, size_t x, size_t y, size_t k)
{
    for (size_t i = 0; i < k; i++) swap_ij(a, x + i, y + i);
}

/*
 * Merging by exchanges (the swap principle of Sec. "QuickXsort and
 * QuickMergesort": an element that Mergesort would write to extra space is
 * exchanged with the buffer element sitting in that cell).
 *
 * The output window W = [w, w + nx + ny) holds buffer elements in its first
 * nx cells and the sorted run Y in its last ny cells; the sorted run X has
 * nx elements at [x0, x0 + nx), outside W.  Each output cell, from the left,
 * is exchanged with the smaller of the two run heads (Y's head on equal
 * keys).  While X is not used up, the cells between the next output cell and
 * Y's head are exactly the not yet displaced buffer elements, so an exchange
 * never moves a run element out of reach.  Once X is used up the rest of Y
 * already lies in place.  Afterwards W holds the nx + ny run elements in
 * order and [x0, x0 + nx) holds the buffer elements (in some order).
 */
static void swap_merge(arr_t *a, size_t x0, size_t nx, size_t w, size_t ny)
{
    const size_t x_end = x0 + nx, w_end = w + nx + ny;
    size_t x = x0, y = w + nx, o = w;
    for (; x < x_end; o++) {
        const int take_y = y < w_end && !less_ij(a, x, y);
        if (take_y) {
            swap_ij(a, o, y);
            y++;
        } else {
            swap_ij(a, o, x);
            x++;
        }
    }
}

static void clever_quicksort(arr_t *a, size_t lo, size_t hi);

/*
 * Mergesort into a disjoint target: the n elements at [src, src + n) end
 * sorted at [dst, dst + n), and the n elements found there end at
 * [src, src + n).  The first h = floor(n/2) and the last k = n - h elements
 * are sorted separately (the last k straight into the tail of the target,
 * the first h into the cells the last k have just vacated, which now hold
 * target elements) and then merged into the target.  Blocks shorter than
 * X_THRESH are sorted by X where they are and exchanged into the target as
 * one block (QuickMergeXsort's joint movement; with X_THRESH = 2 a single
 * element is its own sorted run).  Reading R3 fixes the size of the first
 * run of the merge.
 */
static void sort_to(arr_t *a, size_t src, size_t n, size_t dst)
{
    if (n < a->xt) {
        clever_quicksort(a, src, src + n);
        swap_blocks(a, src, dst, n);
        return;
    }
    const size_t h = n / 2, k = n - h;
    sort_to(a, src + h, k, dst + h);
    sort_to(a, src, h, src + h);
    swap_merge(a, src + h, h, dst, k);
}

/*
 * Mergesort in place: sorts the n elements at [lo, lo + n) with the
 * ceil(n/2) cells at buf as swap space (they get their elements back,
 * permuted).  The last k = ceil(n/2) elements go sorted to the swap space,
 * the first h = floor(n/2) sorted to the top h cells of the range, and the
 * run in the swap space is merged back into the range (Fig. 1 shows this
 * placement).
 */
static void sort_with_buffer(arr_t *a, size_t lo, size_t n, size_t buf)
{
    if (n < 2) return;
    const size_t h = n / 2, k = n - h;
    sort_to(a, lo + h, k, buf);
    sort_to(a, lo, h, lo + k);
    swap_merge(a, buf, k, lo, h);
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

/*
 * QuickMergesort on [lo, hi) (Sec. "QuickXsort and QuickMergesort"):
 * partition around the median of three; the side with fewer than half of
 * the range's elements (reading R2) is mergesorted, the other side serving
 * as its swap space; the other side is what remains to be sorted.
 */
static void quick_merge_sort(arr_t *a, size_t lo, size_t hi)
{
    for (size_t n = hi - lo; n > 2; n = hi - lo) {
        const size_t p = partition(a, lo, hi);
        const size_t n_left = p - lo, n_right = hi - (p + 1);
        if (n_left < n / 2) {
            sort_with_buffer(a, lo, n_left, p + 1);
            lo = p + 1;
        } else {
            sort_with_buffer(a, p + 1, n_right, lo);
            hi = p;
        }
    }
    if (hi - lo == 2) cmp_exchange(a, lo, lo + 1); /* R5 */
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
    quick_merge_sort(&a, 0, n);
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
    quick_merge_sort(&a, 0, n);
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

#if QMSO_COUNTING
static int cmp_key(const void *x, const void *y)
{
    qkey_t a = *(const qkey_t *)x, b = *(const qkey_t *)y;
    return (a > b) - (a < b);
}

/* R7: the median of the floor(n/3) medians of three (MoMQuickMergesort's
 * pivot, Sec. "Worst-Case Efficient QuickMergeSort"), as the key bits of the
 * input (is_f32: compared by R6, binary32 or binary64 by the key width).
 * n >= 3.  Returns 0 and sets *ok = 0 if memory runs out.  Exported from the
 * counting builds as qmso_mom_pivot and qmso64_mom_pivot. */
qkey_t QMSO_FN(mom_pivot)(const qkey_t *keys, size_t n, int is_f32, int *ok)
{
    size_t c = n / 3;
    qkey_t *med = malloc((c ? c : 1) * sizeof(qkey_t));
    *ok = med != NULL && c > 0;
    if (!*ok) {
        free(med);
        return 0;
    }
    for (size_t i = 0; i < c; i++) {
        qkey_t x = keys[3 * i], y = keys[3 * i + 1], z = keys[3 * i + 2];
        if (is_f32) {
            x = f32_bits_to_key(x);
            y = f32_bits_to_key(y);
            z = f32_bits_to_key(z);
        }
        /* median of three: the one that is neither the smallest nor the largest */
        qkey_t lo = x < y ? x : y, hi = x < y ? y : x;
        med[i] = z < lo ? lo : (z > hi ? hi : z);
    }
    qsort(med, c, sizeof(qkey_t), cmp_key);
    qkey_t p = med[(c - 1) / 2];
    free(med);
    return is_f32 ? key_to_f32_bits(p) : p;
}
#endif

#if QMSO_COUNTING && QMSO_KEY_BITS == 32
/* The pieces below are exported only from the counting build, for tests
 * that pin the individual routines: the partition, the Mergesort into a
 * target (msort), the Mergesort with a buffer (out) and the exchange merge
 * (merge), the last three with the argument conventions of Fig. 2.  Keys
 * are plain u32. */

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
    sort_with_buffer(&a, begin, end - begin, temp);
}

void qmso_msort(uint32_t *keys, uint32_t *vals, size_t begin, size_t end,
                size_t target, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    sort_to(&a, begin, end - begin, target);
}

/* the Mergesort into a target with X = CleverQuicksort below x_thresh
 * (QuickMergeXsort) */
void qmso_msort_x(uint32_t *keys, uint32_t *vals, size_t begin, size_t end,
                  size_t target, size_t x_thresh, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch),
               x_thresh < 2 ? 2 : x_thresh};
    sort_to(&a, begin, end - begin, target);
}

void qmso_merge(uint32_t *keys, uint32_t *vals, size_t begin1, size_t end1,
                size_t target, size_t endtarget, qmso_counters *counters)
{
    qmso_counters scratch;
    arr_t a = {keys, vals, counters_or_scratch(counters, &scratch), 2};
    swap_merge(&a, begin1, end1 - begin1, target, endtarget - target - (end1 - begin1));
}
#endif
