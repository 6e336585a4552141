// qms_device.hpp -- device-side building blocks shared by the QuickMergesort
// kernels for gfx950 (CDNA4: 64-lane wavefronts, 160 KB LDS per CU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qms {

// ---- launch geometry and tile sizes -----------------------------------------
constexpr int kBlock = 256;            // threads per workgroup (4 waves)
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kWaves = kBlock / kWave;

// Build-time tunables (defaults are the shipped configuration).
#ifndef QMS_MERGE_ITEMS
#define QMS_MERGE_ITEMS 8
#endif
#ifndef QMS_SPLIT_LANES
#define QMS_SPLIT_LANES 4
#endif

constexpr int kSortThreads = 512;      // threads of the base-case workgroup
constexpr uint32_t kBaseTileKeys = 16384;  // base-case tile, keys only
constexpr uint32_t kBaseTilePairs = 8192;  // base-case tile, key/payload pairs
#ifndef QMS_WIDE_PAIR_TILE
#define QMS_WIDE_PAIR_TILE 2048
#endif
constexpr uint32_t kBaseTileWidePairs = QMS_WIDE_PAIR_TILE;  // 64-bit keys with payloads
// The base tile of a sort: keys only, key/payload pairs or 64-bit keys, or
// 64-bit keys with payloads (whose 128-bit network elements fill the LDS
// four times as fast).
__host__ __device__ constexpr uint32_t base_tile_of(bool pairs, bool wide) {
    return pairs && wide ? kBaseTileWidePairs : (pairs || wide) ? kBaseTilePairs : kBaseTileKeys;
}
constexpr int kMergePerThread = QMS_MERGE_ITEMS;       // outputs per thread
constexpr int kMergeTile = kBlock * kMergePerThread;   // outputs per workgroup
// Run samples: every kSampleStride-th element of every sorted run, written by
// the pass that produced the run; the next pass's split searches start on
// them and finish inside one sample gap of the runs (a smaller stride leaves
// fewer cache lines of the runs to touch there).
#ifndef QMS_SAMPLE_STRIDE
#define QMS_SAMPLE_STRIDE 256
#endif
constexpr uint32_t kSampleStride = QMS_SAMPLE_STRIDE;
constexpr uint32_t kSamplesPerTile = (uint32_t)kMergeTile / kSampleStride;
static_assert((uint32_t)kMergeTile % kSampleStride == 0 && kSampleStride >= 64,
              "samples at a divisor of the merge tile");
constexpr uint32_t kSplitLanes = QMS_SPLIT_LANES;      // lanes per merge-path split
constexpr int kPartSub = 4096;         // elements a workgroup classifies per step
constexpr int kPartItems = kPartSub / kBlock;          // 16
#ifndef QMS_RANK_CHUNK
#define QMS_RANK_CHUNK 2048
#endif
constexpr int kRankChunk = QMS_RANK_CHUNK;  // misplaced pairs exchanged per workgroup
constexpr uint32_t kMaxTiles = 65536;  // fixed bound on partition tiles
constexpr int kScanThreads = 1024;     // block size of the scans of large ranges
constexpr int kScanPer = 8;            // tiles per thread and step of a scan
constexpr uint32_t kScanGroups = 16;   // workgroups per segment of the pass-A scan
constexpr uint64_t kEqBlockMin = 64;   // pivot-equal keys that always get their own block
// Median-of-medians select: triples per histogram workgroup (kBlock threads
// x kMomPerThread), and the workgroups a range of s keys takes.
constexpr int kMomPerThread = 32;
constexpr uint32_t kMomTile = (uint32_t)kBlock * kMomPerThread;
__host__ __device__ inline uint32_t mom_tiles_of(uint64_t s) {
    return (uint32_t)((s / 3 + kMomTile - 1) / kMomTile);
}
// Workgroups of the pass-A scan of a range of nt tiles, scans of nth threads:
// one per chunk of nth * kScanPer tiles, at most kScanGroups.
__host__ __device__ inline uint32_t scan_a_groups(uint32_t nt, uint32_t nth) {
    const uint32_t C = nth * (uint32_t)kScanPer;
    const uint32_t chunks = (nt + C - 1) / C;
    return chunks < kScanGroups ? chunks : kScanGroups;
}

static_assert(kBaseTileKeys % kMergeTile == 0 && kBaseTilePairs % kMergeTile == 0 &&
                  kBaseTileWidePairs % kMergeTile == 0,
              "runs must tile into merge tiles");

// ---- round state slots (uint64 words in the workspace) ----------------------
enum MetaSlot : int {
    M_PIVOT = 0,   // pivot key (order-mapped)
    M_CLT = 1,     // # keys < pivot
    M_CEQ = 2,     // # keys == pivot
    M_XA = 3,      // misplaced pairs of pass A (< pivot vs the rest)
    M_TB = 4,      // tile holding the </>= boundary
    M_LTPART = 5,  // # keys < pivot in that tile, left of the boundary
    M_EQPART = 6,  // # keys == pivot in that tile, left of the boundary
    M_XB = 7,      // misplaced pairs of pass B (== pivot vs > pivot)
    M_RCA = 8,     // misplaced pairs per chunk, pass A
    M_RCB = 9,     // misplaced pairs per chunk, pass B
    M_MOM_PREFIX = 10,  // median-of-medians pivot: digits chosen so far
    M_MOM_RANK = 11,    // median-of-medians pivot: rank inside the prefix
    M_MOM_DONE = 12,    // median-of-medians pivot: histogram workgroups done this pass
    M_COUNT = 16
};

// Misplaced pairs per swap chunk for a pass with X pairs over a range of s
// keys: at most kRankChunk (the LDS slots of a workgroup), and small enough
// that there are about s / span chunks (span >= kPartSub, a tunable; default
// kChunkSpan), so that sparse misplacement (nearly sorted input) still
// spreads the range scans over many workgroups.
constexpr uint64_t kChunkSpan = 4 * kPartSub;  // default target positions per chunk
__host__ __device__ inline uint32_t rank_chunk(uint64_t X, uint64_t s, uint64_t span) {
    const uint64_t target = (s + span - 1) / span;
    uint64_t rc = (X + target - 1) / target;
    if (rc < 1) rc = 1;
    if (rc > (uint64_t)kRankChunk) rc = kRankChunk;
    return (uint32_t)rc;
}
__host__ __device__ inline uint64_t chunk_count(uint64_t X, uint64_t s, uint64_t span) {
    const uint32_t rc = rank_chunk(X, s, span);
    return (X + rc - 1) / rc;
}

// ---- task tables ----------------------------------------------------------------
// A launch serves many independent segments (arrays) at once.  The host lists
// the segments of a phase in a table and gives each a number of work items
// (workgroups or waves); `pre` is the exclusive prefix of those counts, so
// work item g belongs to the segment a with pre[a] <= g < pre[a + 1].  With a
// single segment the table travels by value in the kernel arguments and no
// lookup is done.

// One segment in a partition round: the keys of the range [lo, lo + s).
struct PartSeg {
    uint32_t *keys;      // segment base
    uint32_t *vals;      // payloads (nullptr for keys only)
    uint32_t lo, s;      // current range, relative to keys
    uint32_t tile_off;   // first entry of the segment in the per-tile arrays
    uint32_t nt;         // partition tiles of the range
    uint32_t chunk_off;  // first entry in the chunk-boundary arrays
    uint32_t slot;       // index of the segment's round-state words
    uint32_t flags;      // kPivotMoM: pivot precomputed by the median-of-medians select
    uint32_t pad;        // histogram slot of that select
};
constexpr uint32_t kPivotMoM = 1;

// One Mergesort of a round: m keys in the data region D, m cells of swap
// space in the buffer region Bf (the other side of the partition; a final
// range has L = 0 and no buffer), L merge levels over runs of
// w0 << level keys; the base case swaps into Bf when the pass count is odd.
// The pointers address element 0 of each region (keys of the sort's width).
struct SortSeg {
    uint32_t *keys;      // D
    uint32_t *vals;      // payloads of D (nullptr for keys only)
    uint32_t *bkeys;     // Bf (unused when L == 0)
    uint32_t *bvals;     // payloads of Bf
    uint32_t m;
    uint32_t L;          // merge levels
    uint32_t split_off;  // first entry in the merge split array
    uint32_t w0;         // base-case tile (run width of level 0)
    uint32_t two_way;    // 1: 2-way passes only (key/payload sorts, or by tuning)
    uint32_t pad;
};

// Merge passes of a Mergesort task with L binary levels (runs of w0 << l
// keys after level l).  Key-only tasks merge four runs per pass: a 2-way pass
// first when L is odd, then 4-way passes, ceil(L / 2) passes in all.
// Key/payload tasks run L 2-way passes.  The pass that starts at binary level
// `level` has index pass_index(); passes alternate between the two regions,
// and the base case writes into the buffer exactly when the pass count is
// odd, so that the last pass ends in the data region.
// `two` selects the 2-way schedule (key/payload tasks always; key-only
// tasks by tuning).
__host__ __device__ inline uint32_t merge_passes(uint32_t L, bool two) {
    return two ? L : (L + 1) / 2;
}
__host__ __device__ inline uint32_t pass_index(uint32_t L, uint32_t level, bool two) {
    return two ? level : ((L & 1u) ? (level + 1) / 2 : level / 2);
}

// Two ways to size a launch:
//   host-sized   the host knows the work items and launches exactly that
//                many workgroups (dyn == nullptr): workgroup g takes item g;
//   device-sized the round plan, a kernel, wrote the tables and the number
//                of work items into device memory (*dyn).  The host
//                launches a grid from its estimate of the work: workgroup g
//                takes item g if that is below *dyn, and a second, looping
//                launch of the same kernel (a few workgroups, taking the
//                items from the estimate on in grid-stride order) covers
//                whatever the estimate missed.  The one-item form keeps the
//                registers of the kernel body as they are (a loop around
//                these bodies lets the compiler hoist thread-invariant
//                values out of it and spill).  The prefix then has A + 1
//                entries with every entry past the plan's last segment
//                equal to the total, so that the lookup below never lands
//                on an unused entry.
template <class T>
struct TaskRef {
    const T *tab = nullptr;        // device table (A > 1)
    const uint32_t *pre = nullptr; // device prefix of work items, A + 1 entries (A > 1)
    uint32_t A = 0;                // segments (an upper bound when device-sized)
    uint32_t base = 0;             // pre[0] (a sub-range of a longer table; A > 1)
    T one;               // the segment itself when A == 1
    const uint32_t *dyn = nullptr; // device-sized: the number of work items
    const uint32_t *dyn_A = nullptr;  // device-sized: the number of segments (else A)
};

// Work items of a launch: the plan's count when device-sized, else the
// count the host gives (the items its grid covers).
template <class T>
__device__ __forceinline__ uint32_t work_total(const TaskRef<T> &r, uint32_t host_total) {
    return r.dyn ? *r.dyn : host_total;
}

// Work item g -> segment index (largest a with pre[a] <= g).
__device__ __forceinline__ uint32_t find_task(const uint32_t *pre, uint32_t A, uint32_t g) {
    uint32_t lo = 0, hi = A;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <class T>
__device__ __forceinline__ T task_of(const TaskRef<T> &r, uint32_t g, uint32_t *local,
                                     uint32_t *index) {
    if (r.A == 1) {
        *local = g;
        *index = 0;
        return r.one;
    }
    g += r.base;
    const uint32_t a = find_task(r.pre, r.dyn_A ? *r.dyn_A : r.A, g);
    *local = g - r.pre[a];
    *index = a;
    return r.tab[a];
}

// The same search for a g that every lane of a wave holds, all 64 lanes
// taking part: each step the lanes probe 64 evenly spaced entries of the
// candidate range and a ballot keeps the part after the last probe at or
// below g, so A segments take ceil(log64 A) dependent loads instead of
// ceil(log2 A) (20,000 segments: 3 instead of 15).
__device__ __forceinline__ uint32_t find_task_wave(const uint32_t *pre, uint32_t A, uint32_t g) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t lo = 0, n = A;  // the answer lies in [lo, lo + n); pre[lo] <= g
    while (n > 1) {
        const uint32_t step = (n + 63) / 64;
        const uint32_t off = lane * step;
        const bool ok = off < n && pre[lo + off] <= g;  // a prefix of the lanes
        const uint64_t m = __ballot(ok);
        const uint32_t last = 63u - (uint32_t)__clzll((long long)m);
        lo += last * step;
        const uint32_t rest = n - last * step;
        n = rest < step ? rest : step;
    }
    return lo;
}

template <class T>
__device__ __forceinline__ T task_of_wave(const TaskRef<T> &r, uint32_t g, uint32_t *local,
                                          uint32_t *index) {
    if (r.A == 1) {
        *local = g;
        *index = 0;
        return r.one;
    }
    g += r.base;
    const uint32_t a = find_task_wave(r.pre, r.dyn_A ? *r.dyn_A : r.A, g);
    *local = g - r.pre[a];
    *index = a;
    return r.tab[a];
}

// Per-lane g, non-decreasing with the lane, all 64 lanes taking part: the
// searches for the first and the last lane's g bound every lane's, which
// then searches the few segments between them.
template <class T>
__device__ __forceinline__ T task_of_lanes(const TaskRef<T> &r, uint32_t g, uint32_t *local,
                                           uint32_t *index) {
    if (r.A == 1) {
        *local = g;
        *index = 0;
        return r.one;
    }
    g += r.base;
    const uint32_t A = r.dyn_A ? *r.dyn_A : r.A;
    const uint32_t g0 = (uint32_t)__shfl((int)g, 0), g1 = (uint32_t)__shfl((int)g, 63);
    uint32_t lo = find_task_wave(r.pre, A, g0);
    uint32_t hi = g1 == g0 ? lo + 1 : find_task_wave(r.pre, A, g1) + 1;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (r.pre[mid] <= g) lo = mid;
        else hi = mid;
    }
    *local = g - r.pre[lo];
    *index = lo;
    return r.tab[lo];
}

// ---- key order ----------------------------------------------------------------
// Keys are compared as unsigned integers of their own width (K: 32 or 64
// bits) after an order map applied in registers on load (and undone on
// store).  The policy carries the key type, so kernels templated on it read
// and write keys of the right width.
// lt(a, b) compares two mapped keys; NetKey is the element type of the base
// case's network for keys without payloads.
struct OrdU32 {
    using K = uint32_t;
    using NetKey = uint32_t;
    __device__ __forceinline__ static uint32_t ord(uint32_t x) { return x; }
    __device__ __forceinline__ static uint32_t unord(uint32_t x) { return x; }
    __device__ __forceinline__ static bool lt(uint32_t a, uint32_t b) { return a < b; }
};
// IEEE-754 binary32 total order: negative values have all bits flipped,
// non-negative values get the sign bit set; unsigned order of the result is
// the total order (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN).
struct OrdF32 {
    using K = uint32_t;
    using NetKey = uint32_t;
    __device__ __forceinline__ static bool lt(uint32_t a, uint32_t b) { return a < b; }
    __device__ __forceinline__ static uint32_t ord(uint32_t u) {
        return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
    }
    __device__ __forceinline__ static uint32_t unord(uint32_t k) {
        return k ^ ((uint32_t)((int32_t)(~k) >> 31) | 0x80000000u);
    }
};
// 64-bit keys: unsigned, and IEEE-754 binary64 by the same total order.
struct OrdU64 {
    using K = uint64_t;
    using NetKey = uint64_t;
    __device__ __forceinline__ static bool lt(uint64_t a, uint64_t b) { return a < b; }
    __device__ __forceinline__ static uint64_t ord(uint64_t x) { return x; }
    __device__ __forceinline__ static uint64_t unord(uint64_t x) { return x; }
};
struct OrdF64 {
    using K = uint64_t;
    using NetKey = uint64_t;
    __device__ __forceinline__ static bool lt(uint64_t a, uint64_t b) { return a < b; }
    __device__ __forceinline__ static uint64_t ord(uint64_t u) {
        return u ^ ((uint64_t)((int64_t)u >> 63) | 0x8000000000000000ull);
    }
    __device__ __forceinline__ static uint64_t unord(uint64_t k) {
        return k ^ ((uint64_t)((int64_t)(~k) >> 63) | 0x8000000000000000ull);
    }
};
// An expensive comparison (the paper's Experiments section sorts integers
// with a comparator that applies the logarithm to them): uint32 keys
// ordered by log(key) in double precision, evaluated at every comparison.
// log is strictly increasing and double precision separates the logarithms
// of any two distinct integers below 2^32 (their gap is at least about
// 2^-32, the spacing of doubles near 22 is 2^-48), so the order is the
// integers' own (log 0 = -inf comes first) and the sorted output is the
// plain uint32 sort.  Equality is integer equality.
__device__ __forceinline__ bool log_less(uint32_t a, uint32_t b) {
    return log((double)a) < log((double)b);
}
// The network element of that order: the complement still reverses it
// (any order-reversing map of the integers reverses an increasing function
// of them), so the base case's descending-block representation holds.
struct LogKey {
    uint32_t k;
};
__device__ __forceinline__ bool operator<(LogKey a, LogKey b) { return log_less(a.k, b.k); }
__device__ __forceinline__ LogKey operator^(LogKey a, LogKey b) { return LogKey{a.k ^ b.k}; }
__device__ __forceinline__ LogKey &operator^=(LogKey &a, LogKey b) {
    a.k ^= b.k;
    return a;
}
struct OrdLogU32 {
    using K = uint32_t;
    using NetKey = LogKey;
    __device__ __forceinline__ static uint32_t ord(uint32_t x) { return x; }
    __device__ __forceinline__ static uint32_t unord(uint32_t x) { return x; }
    __device__ __forceinline__ static bool lt(uint32_t a, uint32_t b) { return log_less(a, b); }
};

// The largest key of a width (the merge sentinel, the base case's padding).
template <class K>
__device__ __forceinline__ constexpr K key_max() { return ~K(0); }

// ---- global memory access -------------------------------------------------------
// Pointers taken from task tables are generic; accessing them through the
// global address space lets the compiler emit global_load/store (not flat).
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) uint64_t g_u64;
__device__ __forceinline__ uint32_t ldg(const uint32_t *p) { return *(const g_u32 *)p; }
__device__ __forceinline__ void stg(uint32_t *p, uint32_t v) { *(g_u32 *)p = v; }
__device__ __forceinline__ uint64_t ldg(const uint64_t *p) { return *(const g_u64 *)p; }
__device__ __forceinline__ void stg(uint64_t *p, uint64_t v) { *(g_u64 *)p = v; }

// ---- wave and block primitives -------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x / kWave); }
__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(v, d, kWave);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive scan over the whole block; `tmp` holds >= blockDim/64 + 1 words
// of LDS.  Returns the prefix; *total gets the block sum.  Every thread of
// the block must call it.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *tmp, T *total) {
    const int lane = lane_id(), wave = wave_id();
    const int nwaves = (int)(blockDim.x / kWave);
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) tmp[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        T w = lane < nwaves ? tmp[lane] : T(0);
        T wi = wave_inclusive_scan(w);
        if (lane < nwaves) tmp[lane] = wi - w;
        if (lane == nwaves - 1) tmp[nwaves] = wi;
    }
    __syncthreads();
    T res = tmp[wave] + inc - v;
    *total = tmp[nwaves];
    __syncthreads();
    return res;
}

template <class T>
__device__ __forceinline__ T block_sum(T v, T *tmp) {
    T total;
    (void)block_exclusive_scan(v, tmp, &total);
    return total;
}

__device__ __forceinline__ uint32_t median3(uint32_t a, uint32_t b, uint32_t c) {
    return max(min(a, b), min(max(a, b), c));
}
__device__ __forceinline__ uint64_t median3(uint64_t a, uint64_t b, uint64_t c) {
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    const uint64_t m = hi < c ? hi : c;
    return lo > m ? lo : m;
}

// Median of three order-mapped keys by the policy's comparison (three
// comparisons, as Theorem 1's proof charges; for the integer orders the same
// value as median3).
template <class O>
__device__ __forceinline__ typename O::K median3_by(typename O::K a, typename O::K b,
                                                    typename O::K c) {
    using K = typename O::K;
    const bool ba = O::lt(b, a);
    const K lo = ba ? b : a, hi = ba ? a : b;
    const K m = O::lt(c, hi) ? c : hi;
    return O::lt(m, lo) ? lo : m;
}

// Pivot of the range [lo, hi): median of the keys at lo, lo + s/2 and hi - 1.
template <class O>
__device__ __forceinline__ typename O::K pivot_of(const typename O::K *keys, uint64_t lo,
                                                  uint64_t hi) {
    const uint64_t s = hi - lo;
    return median3_by<O>(O::ord(ldg(keys + lo)), O::ord(ldg(keys + lo + s / 2)),
                         O::ord(ldg(keys + hi - 1)));
}

}  // namespace qms
