// qms_rounds.hip -- the QuickMergesort loop of a batch with its round
// control on the device: no host readback, no stream synchronisation, so a
// whole batch can be enqueued at once (and captured in a HIP graph).
//
// The host-driven loop (qms_driver.cpp) reads three counters per segment
// back after each partition count to size the rest of the round.  Here the
// segment states (range, pivot rule, whether a range waits for the base
// case) stay in device memory, and small single-workgroup plan kernels turn
// them into the task tables of each phase: the partition table and its tile
// and scan prefixes before the count, the exchange chunks after the scan,
// the side choice (Fig. 2 sort(): the smaller side is mergesorted with the
// larger side as swap space, the loop keeps the larger one) and the
// Mergesort tasks with their tile and pass prefixes.  The phase kernels are
// the same as the host-driven loop's; they read their work-item counts from
// device memory and take their items in grid-stride order, so the host only
// has to launch an upper bound of workgroups.
//
// The host enqueues a fixed schedule for the batch: R rounds with
// HybridQuickMergesort's pivot rule (Sec. "Worst-Case Efficient
// QuickMergeSort": median-of-3, or after a round whose smaller side held
// less than 1/16 of its range the median of the medians of three), then X
// at the loop level: every range still above the base tile is sorted in
// place by the bitonic network of qms_bitonic.hip (its tiles by the base
// case first), as the host-driven loop finishes its last range.  R covers
// 1.2 rounds per binary level between the longest segment and the loop's
// exit size (plus two), so with random keys the network has little left;
// its passes are enqueued for the largest range the rule allows and read
// zero counts when nothing is left, as do the rounds' launches.  Upper
// bounds for the launch sizes, the merge passes and the network follow from
// the same rule: a range shrinks by 1/16 in a round with a balanced split,
// and after an unbalanced round the median-of-medians round removes a
// third, so after r >= 1 rounds a range of n keys holds at most
// n (15/16)^(r-1) keys.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "qms.h"
#include "qms_device.hpp"
#include "qms_host.hpp"
#include "qms_internal.hpp"

namespace qms {

namespace {

constexpr int kPlanThreads = 1024;
// Segment flags.
constexpr uint32_t DS_ACTIVE = 1;  // range above the base tile: partitioned this round
constexpr uint32_t DS_MOM = 2;     // next pivot: median of the medians of three
constexpr uint32_t DS_FINAL = 4;   // range of at most the base tile: base case next round
constexpr uint32_t DS_NET = 8;     // range left the loop (at most F keys): network at the end

// Workspace counters (dwork) of the device-sized launches of a round.
enum WorkSlot : int {
    W_ACTIVE = 0,  // segments in the partition table
    W_TILES,       // partition tiles
    W_SCAN,        // pass-A scan workgroups
    W_MOM,         // median-of-medians histogram tiles
    W_SPLIT_A,     // split waves, pass A
    W_SWAP_A,      // exchange chunks, pass A
    W_SPLIT_B,
    W_SWAP_B,
    W_SORT_TASKS,  // Mergesort tasks
    W_BASE,        // base-case tiles
    W_MERGE2,      // merge tiles of the 2-way first passes
    W_STEP0,       // merge tiles of 4-way (or 2-way) step k: W_STEP0 + k
    W_ERRORS = W_STEP0 + kMaxLevels,  // inconsistent counts, passes beyond the schedule
    W_LEFT,        // segments still in the loop at the end of the schedule
    W_LIVE,        // entries of the live list the next round reads
    W_MOM_SEGS,    // segments in the median-of-medians table
    W_COUNT_SLOTS
};
static_assert(W_COUNT_SLOTS <= 64, "work counters fit their array");

struct DevSeg {
    uint32_t *keys, *vals;  // segment base
    uint32_t lo, hi;        // current range, relative to the base
    uint32_t flags;
    uint32_t slot;          // partition slot of the round (active segments)
};

// Round constants shared by the plan kernels.
struct PlanArgs {
    uint32_t nseg;       // segments of the group
    uint32_t TP;         // partition tile
    uint32_t scan_nth;   // threads of the pass-A scan
    uint32_t span;       // exchange-chunk span
    uint32_t T0;         // base tile: ranges of at most T0 keys go to the base case
    uint32_t R0;         // Mergesort run width (X_THRESH)
    uint32_t auto_r0;    // automatic X_THRESH: halve R0 when that makes L even
    uint32_t four_way;   // 4-way passes (else 2-way)
    uint32_t wide;       // 64-bit keys
    uint32_t ew;         // 32-bit words per key
    uint32_t F;          // loop exit: a range of at most F keys (> T0) waits for the network
    uint32_t xfinal;     // the last round: every range above the base tile goes to the network
    uint32_t partitioned;  // this round ran a partition (else only finals are sorted)
    uint32_t steps;      // merge steps enqueued this round
    uint32_t first2;     // a launch for 2-way first passes (odd level counts) is enqueued
    uint32_t cap_tiles, cap_chunks, cap_splits;
};

struct PlanPtrs {
    DevSeg *seg;
    uint32_t *aseg;                // active index -> segment
    // the segments still in the loop (active, or waiting for the base case),
    // compacted by each round's side kernel; nullptr in: every segment
    const uint32_t *live_in;
    uint32_t *live_out;
    PartSeg *ptab, *mtab;
    SortSeg *stab;
    uint32_t *p_tiles, *p_scan, *p_mom, *p_wa, *p_ca, *p_wb, *p_cb, *p_base, *p_m2;
    uint32_t *p_step;              // kMaxLevels arrays of (nseg + 2) entries
    uint32_t *work;
    uint64_t *meta;
    const uint32_t *res;
};

__device__ __forceinline__ uint32_t ceil_log2_dev(uint64_t x) {
    uint32_t l = 0;
    while ((1ull << l) < x) ++l;
    return l;
}

// Block-wide exclusive scan of one value per thread with a running carry
// across the chunks of a loop; returns the prefix, adds the chunk's total to
// *carry (uniform).  Every thread of the block calls it.
__device__ __forceinline__ uint32_t scan_carry(uint32_t v, uint32_t *tmp, uint32_t *carry) {
    uint32_t total;
    const uint32_t pre = block_exclusive_scan(v, tmp, &total) + *carry;
    *carry += total;
    return pre;
}

// ---- init: segment states from the offsets ------------------------------------------
// offsets == nullptr: one segment of single_n keys (a single array).
__global__ __launch_bounds__(kBlock) void k_rounds_init(DevSeg *seg, const uint64_t *offsets,
                                                        uint64_t single_n, uint32_t j0,
                                                        uint32_t nseg, uint32_t *keys_base,
                                                        uint32_t *vals_base, uint32_t ew,
                                                        uint32_t T0, uint32_t *work) {
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < nseg; i += gridDim.x * kBlock) {
        const uint64_t a = offsets ? offsets[j0 + i] : 0, b = offsets ? offsets[j0 + i + 1] : single_n;
        const uint64_t n = b - a;
        DevSeg d;
        d.keys = keys_base + ew * a;
        d.vals = vals_base ? vals_base + a : nullptr;
        d.lo = 0;
        d.hi = (uint32_t)n;
        d.flags = n > T0 ? DS_ACTIVE : (n > 1 ? DS_FINAL : 0u);
        d.slot = 0;
        seg[i] = d;
    }
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < W_COUNT_SLOTS; i += kBlock) work[i] = 0;
}

// ---- plans over many workgroups ------------------------------------------------------
// A plan gives every entry of a list (the live segments, the partition
// slots) its offsets in a phase's tables: exclusive prefixes of a few counts
// per entry.  It takes two launches of kPB-thread workgroups, one entry per
// thread: the first writes each workgroup's sums into blk, the second adds
// the sums of the workgroups before its own to a workgroup scan and writes
// the tables.  Whatever the plan reads from the round's counters is read by
// the first launch and kept in blk's header, since the second launch's first
// workgroup rewrites those counters.  (One 1,024-thread workgroup walking
// all entries took 40 to 75 us per plan on 20,000 segments, most of it
// dependent loads and register spills.)
constexpr int kPlanWaves = kPlanThreads / kWave;
constexpr int kPB = 256;
constexpr int kPBWaves = kPB / kWave;
constexpr uint32_t kPlanBlocks = (kCapSegs + kPB - 1) / kPB;
constexpr uint32_t kBlkStride = 32;  // values per workgroup (header first)
enum BlkHeader { BH_N = 0, BH_OK };

// Exclusive scan across the block (thread order) of the first n <= N of
// the N values of every thread; v gets the prefixes, tot the block totals.
// lds: N * WAVES words.  Every thread of the block calls it.
template <int N, int WAVES>
__device__ __forceinline__ void block_scan_n(uint32_t (&v)[N], uint32_t (&tot)[N], uint32_t n,
                                             uint32_t *lds) {
    const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t inc[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        inc[i] = 0;
        if ((uint32_t)i < n) {
            inc[i] = wave_inclusive_scan(v[i]);
            if (lane == kWave - 1) lds[i * WAVES + wave] = inc[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        uint32_t before = 0, all = 0;
        if ((uint32_t)i < n) {
            for (uint32_t w = 0; w < (uint32_t)WAVES; ++w) {
                const uint32_t t = lds[i * WAVES + w];
                before += w < wave ? t : 0u;
                all += t;
            }
        }
        v[i] = (uint32_t)i < n ? before + inc[i] - v[i] : 0u;
        tot[i] = all;
    }
    __syncthreads();  // the LDS may be reused
}

// The block [*a0, *a1) of a list of `count` entries that this thread of a
// kPlanThreads workgroup owns (one-workgroup plans).
__device__ __forceinline__ void owned_block(uint32_t count, uint32_t *a0, uint32_t *a1) {
    const uint32_t per = (count + kPlanThreads - 1) / kPlanThreads;
    const uint32_t b = threadIdx.x * per;
    *a0 = b < count ? b : count;
    *a1 = b + per < count ? b + per : count;
}

// First launch of a plan: this workgroup's sums of the first n <= N counts.
template <int N>
__device__ __forceinline__ void plan_block_sums(uint32_t (&c)[N], uint32_t n, uint32_t *blk,
                                                uint32_t *lds) {
    uint32_t tot[N];
    block_scan_n<N, kPBWaves>(c, tot, n, lds);
    if (threadIdx.x == 0)
        for (uint32_t i = 0; i < n; ++i) blk[(blockIdx.x + 1) * kBlkStride + i] = tot[i];
}

// Second launch: the sums of the nblk workgroups' first n counts before this
// one (base) and over all of them (tot).  sh: kPlanBlocks * kBlkStride words.
template <int N>
__device__ __forceinline__ void plan_block_bases(const uint32_t *blk, uint32_t nblk, uint32_t n,
                                                 uint32_t (&base)[N], uint32_t (&tot)[N],
                                                 uint32_t *sh) {
    for (uint32_t q = threadIdx.x; q < nblk * kBlkStride; q += kPB) sh[q] = blk[kBlkStride + q];
    __syncthreads();
    uint32_t mb = 0, mt = 0;
    if (threadIdx.x < n)
        for (uint32_t q = 0; q < nblk; ++q) {
            const uint32_t v = sh[q * kBlkStride + threadIdx.x];
            mb += q < blockIdx.x ? v : 0u;
            mt += v;
        }
    __syncthreads();
    if (threadIdx.x < n) {
        sh[threadIdx.x] = mb;
        sh[kBlkStride + threadIdx.x] = mt;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        base[i] = (uint32_t)i < n ? sh[i] : 0u;
        tot[i] = (uint32_t)i < n ? sh[kBlkStride + i] : 0u;
    }
    __syncthreads();  // sh may be reused
}

// ---- plan of the partition: table, tile / scan / median-of-medians prefixes ----------
// Counts of one segment: partition slot, tiles, pass-A scan workgroups,
// exchange chunks, median-of-medians slot, its histogram tiles.
enum PlanVal { PV_ACT = 0, PV_TILES, PV_SCAN, PV_CHUNK, PV_MOM, PV_MOM_TILES, PV_N };

__device__ __forceinline__ void plan_counts(const PlanArgs &A, const DevSeg &d,
                                            uint32_t (&c)[PV_N]) {
    const bool act = (d.flags & DS_ACTIVE) != 0;
    const uint32_t s = act ? d.hi - d.lo : 0;
    const uint32_t nt = act ? (s + A.TP - 1) / A.TP : 0;
    const bool mom = act && (d.flags & DS_MOM) != 0;
    c[PV_ACT] = act ? 1u : 0u;
    c[PV_TILES] = nt;
    c[PV_SCAN] = act ? scan_a_groups(nt, A.scan_nth) : 0u;
    c[PV_CHUNK] = act ? (s + 4095) / 4096 + 2 : 0u;
    c[PV_MOM] = mom ? 1u : 0u;
    c[PV_MOM_TILES] = mom ? mom_tiles_of(s) : 0u;
}

__global__ __launch_bounds__(kPB) void k_rounds_plan_count(PlanArgs A, PlanPtrs P,
                                                            uint32_t *blk) {
    __shared__ uint32_t lds[PV_N * kPBWaves];
    const uint32_t n = P.live_in ? P.work[W_LIVE] : A.nseg;
    if (blockIdx.x == 0 && threadIdx.x == 0) blk[BH_N] = n;
    if (blockIdx.x * kPB >= n) return;
    const uint32_t a = blockIdx.x * kPB + threadIdx.x;
    uint32_t c[PV_N] = {};
    if (a < n) plan_counts(A, P.seg[P.live_in ? P.live_in[a] : a], c);
    plan_block_sums<PV_N>(c, PV_N, blk, lds);
}

__global__ __launch_bounds__(kPB) void k_rounds_plan_write(PlanArgs A, PlanPtrs P,
                                                            const uint32_t *blk) {
    __shared__ uint32_t lds[PV_N * kPBWaves];
    __shared__ uint32_t sh[kPlanBlocks * kBlkStride];
    const uint32_t n = blk[BH_N];
    const uint32_t nblk = (n + kPB - 1) / kPB;
    if (blockIdx.x != 0 && blockIdx.x >= nblk) return;
    uint32_t base[PV_N], tot[PV_N];
    plan_block_bases<PV_N>(blk, nblk, PV_N, base, tot, sh);
    const uint32_t a = blockIdx.x * kPB + threadIdx.x;
    uint32_t jj = 0, c[PV_N] = {}, off[PV_N], t2[PV_N];
    DevSeg d{};
    if (a < n) {
        jj = P.live_in ? P.live_in[a] : a;
        d = P.seg[jj];
        plan_counts(A, d, c);
    }
#pragma unroll
    for (int i = 0; i < PV_N; ++i) off[i] = c[i];
    block_scan_n<PV_N, kPBWaves>(off, t2, PV_N, lds);
#pragma unroll
    for (int i = 0; i < PV_N; ++i) off[i] += base[i];
    if (a < n && c[PV_ACT]) {
        const uint32_t ia = off[PV_ACT], im = off[PV_MOM];
        const uint32_t s = d.hi - d.lo;
        const PartSeg pg{d.keys, d.vals, d.lo, s, off[PV_TILES], c[PV_TILES], off[PV_CHUNK], ia,
                         c[PV_MOM] ? kPivotMoM : 0u, im};
        P.ptab[ia] = pg;
        P.aseg[ia] = jj;
        P.seg[jj].slot = ia;
        P.p_tiles[ia] = off[PV_TILES];
        P.p_scan[ia] = off[PV_SCAN];
        if (c[PV_MOM]) {
            P.mtab[im] = pg;
            P.p_mom[im] = off[PV_MOM_TILES];
            uint64_t *meta = P.meta + (uint64_t)ia * M_COUNT;
            const uint64_t cm = s / 3;
            meta[M_MOM_RANK] = (cm - 1) / 2;
            meta[M_MOM_PREFIX] = 0;
            meta[M_MOM_DONE] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t c_act = tot[PV_ACT], c_mom = tot[PV_MOM];
        // a padding entry that no item reaches
        const PartSeg none{nullptr, nullptr, 0, 0, 0, 0, 0, 0, 0, 0};
        P.ptab[c_act] = none;
        P.mtab[c_mom] = none;
        const bool fits = tot[PV_TILES] <= A.cap_tiles && tot[PV_CHUNK] <= A.cap_chunks;
        P.work[W_ACTIVE] = c_act;
        P.work[W_MOM_SEGS] = c_mom;
        P.work[W_TILES] = fits ? tot[PV_TILES] : 0u;
        P.work[W_SCAN] = fits ? tot[PV_SCAN] : 0u;
        P.work[W_MOM] = fits ? tot[PV_MOM_TILES] : 0u;
        if (!fits) atomicAdd(&P.work[W_ERRORS], 1u);
    }
}

// ---- plan of the exchanges: chunks of pass A, bounds of pass B ---------------------
enum SwapVal { SV_WA = 0, SV_CA, SV_WB, SV_CB, SV_BAD, SV_N };

__device__ __forceinline__ void swap_counts(const PlanArgs &A, uint64_t s, uint64_t c_lt,
                                            uint64_t c_eq, uint64_t X, uint32_t (&c)[SV_N]) {
#pragma unroll
    for (int i = 0; i < SV_N; ++i) c[i] = 0;
    if ((c_eq == 0 && c_lt == 0) || c_lt + c_eq > s) {
        c[SV_BAD] = 1;
        return;
    }
    const uint64_t nch = chunk_count(X, s, A.span);
    c[SV_CA] = (uint32_t)nch;
    c[SV_WA] = nch > 1 ? (uint32_t)(2 * (nch - 1)) : 0u;
    // pass B pairs are at most min(#==, #>)
    const uint64_t gt = s - c_lt - c_eq;
    const uint64_t xb = c_eq < gt ? c_eq : gt;
    if (xb > 0) {
        const uint64_t full = (xb + kRankChunk - 1) / kRankChunk;
        const uint64_t target = (s + A.span - 1) / A.span;
        const uint64_t nb = std::min<uint64_t>(xb, std::max(full, target));
        c[SV_CB] = (uint32_t)nb;
        c[SV_WB] = nb > 1 ? (uint32_t)(2 * (nb - 1)) : 0u;
    }
}

__device__ __forceinline__ void swap_counts_of(const PlanArgs &A, const PlanPtrs &P, uint32_t a,
                                               uint32_t (&c)[SV_N]) {
    swap_counts(A, P.ptab[a].s, P.res[4 * a], P.res[4 * a + 1], P.res[4 * a + 2], c);
}

__global__ __launch_bounds__(kPB) void k_rounds_swap_count(PlanArgs A, PlanPtrs P,
                                                            uint32_t *blk) {
    __shared__ uint32_t lds[SV_N * kPBWaves];
    const uint32_t act = P.work[W_ACTIVE];
    const bool ok = P.work[W_TILES] != 0 || act == 0;
    const uint32_t n = ok ? act : 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) blk[BH_N] = n;
    if (blockIdx.x * kPB >= n) return;
    const uint32_t a = blockIdx.x * kPB + threadIdx.x;
    uint32_t c[SV_N] = {};
    if (a < n) swap_counts_of(A, P, a, c);
    plan_block_sums<SV_N>(c, SV_N, blk, lds);
}

__global__ __launch_bounds__(kPB) void k_rounds_swap_write(PlanArgs A, PlanPtrs P,
                                                            const uint32_t *blk) {
    __shared__ uint32_t lds[SV_N * kPBWaves];
    __shared__ uint32_t sh[kPlanBlocks * kBlkStride];
    const uint32_t n = blk[BH_N];
    const uint32_t nblk = (n + kPB - 1) / kPB;
    if (blockIdx.x != 0 && blockIdx.x >= nblk) return;
    uint32_t base[SV_N], tot[SV_N];
    plan_block_bases<SV_N>(blk, nblk, SV_N, base, tot, sh);
    const uint32_t a = blockIdx.x * kPB + threadIdx.x;
    uint32_t c[SV_N] = {}, off[SV_N], t2[SV_N];
    if (a < n) swap_counts_of(A, P, a, c);
#pragma unroll
    for (int i = 0; i < SV_N; ++i) off[i] = c[i];
    block_scan_n<SV_N, kPBWaves>(off, t2, SV_N, lds);
    if (a < n) {
        P.p_wa[a] = base[SV_WA] + off[SV_WA];
        P.p_ca[a] = base[SV_CA] + off[SV_CA];
        P.p_wb[a] = base[SV_WB] + off[SV_WB];
        P.p_cb[a] = base[SV_CB] + off[SV_CB];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.work[W_SPLIT_A] = tot[SV_WA];
        P.work[W_SWAP_A] = tot[SV_CA];
        P.work[W_SPLIT_B] = tot[SV_WB];
        P.work[W_SWAP_B] = tot[SV_CB];
        if (tot[SV_BAD]) atomicAdd(&P.work[W_ERRORS], 1u);
    }
}

// ---- side choice and the Mergesort tasks -------------------------------------------
// For every segment partitioned this round: the smaller of the < and > sides
// is the data region D, m cells of the other side next to the pivot block are
// its buffer; the loop keeps the larger side (Fig. 2 sort()).  A kept range
// of at most T0 keys waits for the base case, which runs in the next round's
// sort launches (it still holds this round's buffer).  Segments whose range
// waited since the last round get their base-case task now.  The segments
// left in the loop form the next round's live list.
enum SideVal { SD_TASK = 0, SD_BASE, SD_SPLIT, SD_M2, SD_LIVE, SD_BAD, SD_STEP0, SD_N = SD_STEP0 + kMaxLevels };

struct SideOut {
    DevSeg d;     // the segment's new state
    SortSeg t;    // its Mergesort (or base-case) task, if emit
    bool emit;
    bool write;   // d changed
};

__device__ __forceinline__ SideOut side_of(const PlanArgs &A, const PlanPtrs &P, DevSeg d,
                                           bool ok, uint32_t lt_eq[2], uint32_t (&c)[SD_N]) {
    SideOut o{};
    o.d = d;
    SortSeg &t = o.t;
    const uint64_t ew = A.ew;
    uint32_t bad = 0;
    if ((d.flags & DS_ACTIVE) && ok) {
        const uint32_t s = d.hi - d.lo;
        const uint32_t c_lt = lt_eq[0], c_eq = lt_eq[1];
        const uint32_t b1 = d.lo + c_lt, b2 = b1 + c_eq;
        const uint32_t mL = c_lt, mR = d.hi - b2;
        o.write = true;
        if ((c_eq == 0 && c_lt == 0) || (uint64_t)c_lt + c_eq > s) {
            // inconsistent counts (the exchange plan skipped this range
            // too): leave the segment, report it
            ++bad;
            o.d.flags = 0;
        } else {
            if (mL <= mR) {
                t.keys = d.keys + ew * d.lo;
                t.vals = d.vals ? d.vals + d.lo : nullptr;
                t.bkeys = d.keys + ew * b2;
                t.bvals = d.vals ? d.vals + b2 : nullptr;
                t.m = mL;
                o.d.lo = b2;
            } else {
                t.keys = d.keys + ew * b2;
                t.vals = d.vals ? d.vals + b2 : nullptr;
                t.bkeys = d.keys + ew * (b1 - mR);
                t.bvals = d.vals ? d.vals + (b1 - mR) : nullptr;
                t.m = mR;
                o.d.hi = b1;
            }
            // run width and levels (as the host-driven loop sets them)
            t.w0 = A.R0;
            t.L = t.m > A.R0 ? ceil_log2_dev((t.m + A.R0 - 1) / A.R0) : 0;
            if (A.auto_r0 && A.four_way && !A.wide && (t.L & 1u)) {
                t.w0 = A.R0 / 2;
                t.L = t.m > t.w0 ? ceil_log2_dev((t.m + t.w0 - 1) / t.w0) : 0;
            }
            t.two_way = A.four_way ? 0u : 1u;
            o.emit = t.m > 1;
            // HybridQuickMergesort, delta = 1/16: an unbalanced split makes
            // the next pivot the median of the medians of three
            const bool unbalanced = (uint64_t)(mL < mR ? mL : mR) * 16 < s;
            const uint32_t s2 = o.d.hi - o.d.lo;
            o.d.flags = s2 > A.F    ? (DS_ACTIVE | (unbalanced ? DS_MOM : 0u))
                        : s2 > A.T0 ? DS_NET
                        : s2 > 1    ? DS_FINAL
                                    : 0u;
        }
    } else if ((d.flags & DS_FINAL) || (A.xfinal && (d.flags & (DS_ACTIVE | DS_NET)))) {
        // the base case in place on the whole remaining range (on each of
        // its tiles for a range the network then finishes)
        t.keys = d.keys + ew * d.lo;
        t.vals = d.vals ? d.vals + d.lo : nullptr;
        t.m = d.hi - d.lo;
        t.L = 0;
        t.w0 = A.T0;
        o.emit = true;
        o.d.flags = 0;
        o.write = true;
    }
    const uint32_t steps_needed = !o.emit ? 0u : t.two_way ? t.L : t.L / 2;  // 4-way passes after the first
    bad += o.emit && steps_needed > A.steps;
    bad += o.emit && !t.two_way && (t.L & 1u) && !A.first2;
    const uint32_t mt = o.emit ? (t.m + kMergeTile - 1) / kMergeTile : 0u;
    c[SD_TASK] = o.emit ? 1u : 0u;
    c[SD_BASE] = o.emit ? (t.m + A.T0 - 1) / A.T0 : 0u;
    c[SD_SPLIT] = t.L ? mt : 0u;  // run samples: Mergesort tasks only
    // the 2-way first pass of a 4-way Mergesort with an odd level count
    c[SD_M2] = o.emit && !t.two_way && (t.L & 1u) ? mt : 0u;
    c[SD_LIVE] = o.d.flags != 0 ? 1u : 0u;
    c[SD_BAD] = bad;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) c[SD_STEP0 + k] = (uint32_t)k < steps_needed ? mt : 0u;
    return o;
}

// One live entry: its segment, and its < p and == p counts when it was
// partitioned this round.
__device__ __forceinline__ void side_load(const PlanPtrs &P, uint32_t a, bool ok, uint32_t *jj,
                                          DevSeg *d, uint32_t (&le)[2]) {
    *jj = P.live_in ? P.live_in[a] : a;
    *d = P.seg[*jj];
    le[0] = le[1] = 0;
    if ((d->flags & DS_ACTIVE) && ok) {
        le[0] = P.res[4 * d->slot];
        le[1] = P.res[4 * d->slot + 1];
    }
}

__global__ __launch_bounds__(kPB) void k_rounds_side_count(PlanArgs A, PlanPtrs P,
                                                            uint32_t *blk) {
    __shared__ uint32_t lds[SD_N * kPBWaves];
    // with no partition this round, or one whose plan did not fit, ranges in
    // the loop stay as they are
    const bool ok = A.partitioned && (P.work[W_TILES] != 0 || P.work[W_ACTIVE] == 0);
    const uint32_t n = P.live_in ? P.work[W_LIVE] : A.nseg;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        blk[BH_N] = n;
        blk[BH_OK] = ok ? 1u : 0u;
    }
    if (blockIdx.x * kPB >= n) return;
    const uint32_t a = blockIdx.x * kPB + threadIdx.x;
    uint32_t c[SD_N] = {};
    if (a < n) {
        uint32_t jj, le[2];
        DevSeg d;
        side_load(P, a, ok, &jj, &d, le);
        (void)side_of(A, P, d, ok, le, c);
    }
    plan_block_sums<SD_N>(c, SD_STEP0 + A.steps, blk, lds);
}

__global__ __launch_bounds__(kPB) void k_rounds_side_write(PlanArgs A, PlanPtrs P,
                                                            const uint32_t *blk) {
    __shared__ uint32_t lds[SD_N * kPBWaves];
    __shared__ uint32_t sh[kPlanBlocks * kBlkStride];
    const uint32_t n = blk[BH_N];
    const bool ok = blk[BH_OK] != 0;
    const uint32_t nblk = (n + kPB - 1) / kPB;
    if (blockIdx.x != 0 && blockIdx.x >= nblk) return;
    const uint32_t nv = SD_STEP0 + A.steps;  // values to scan
    uint32_t base[SD_N], tot[SD_N];
    plan_block_bases<SD_N>(blk, nblk, nv, base, tot, sh);
    const uint32_t a = blockIdx.x * kPB + threadIdx.x;
    uint32_t jj = 0, c[SD_N] = {}, off[SD_N], t2[SD_N];
    SideOut o{};
    if (a < n) {
        uint32_t le[2];
        DevSeg d;
        side_load(P, a, ok, &jj, &d, le);
        o = side_of(A, P, d, ok, le, c);
    }
#pragma unroll
    for (int i = 0; i < SD_N; ++i) off[i] = c[i];
    block_scan_n<SD_N, kPBWaves>(off, t2, nv, lds);
#pragma unroll
    for (int i = 0; i < SD_N; ++i) off[i] += base[i];
    if (a < n) {
        if (o.write) P.seg[jj] = o.d;
        if (c[SD_LIVE]) P.live_out[off[SD_LIVE]] = jj;
        if (o.emit) {
            const uint32_t idx = off[SD_TASK];
            SortSeg t = o.t;
            t.split_off = off[SD_SPLIT];
            P.stab[idx] = t;
            P.p_base[idx] = off[SD_BASE];
            P.p_m2[idx] = off[SD_M2];
#pragma unroll
            for (uint32_t k = 0; k < (uint32_t)kMaxLevels; ++k)
                if (k < A.steps) P.p_step[k * (A.nseg + 2) + idx] = off[SD_STEP0 + k];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t c_task = tot[SD_TASK];
        SortSeg none{};
        P.stab[c_task] = none;
        const bool fits = tot[SD_SPLIT] <= A.cap_splits;
        P.work[W_SORT_TASKS] = c_task;
        P.work[W_BASE] = fits ? tot[SD_BASE] : 0u;
        P.work[W_MERGE2] = fits ? tot[SD_M2] : 0u;
#pragma unroll
        for (uint32_t k = 0; k < (uint32_t)kMaxLevels; ++k)
            if (k < A.steps) P.work[W_STEP0 + k] = fits ? tot[SD_STEP0 + k] : 0u;
        if (!fits || tot[SD_BAD]) atomicAdd(&P.work[W_ERRORS], 1u);
        P.work[W_LIVE] = tot[SD_LIVE];
        // the next round's plan starts from clean counts
        P.work[W_TILES] = 0;
        P.work[W_ACTIVE] = 0;
    }
}

// ---- the network after the last round --------------------------------------------
// The last round's side kernel left one base-case task (L = 0) per range
// still to sort; those above the base tile need the network's passes.  Per
// pass: the work items of every task (bitonic_items_of; zero for the stages
// above a range's own size) and their exclusive prefix, the tables the pass
// kernels search.  A range above 2^K keys, which the schedule's bound rules
// out, is reported as a plan error.
struct NetArgs {
    uint32_t K;   // the network's last stage
    uint32_t T;   // base tile
    uint32_t np;  // passes
    uint32_t PS;  // stride of the prefix arrays
    uint32_t pass[kMaxNetPasses];  // bitonic_passes(): kind | k << 8 | lo << 16 | hi << 24
};
constexpr int kNetBatch = 8;  // passes scanned together

__global__ __launch_bounds__(kPlanThreads) void k_rounds_net_plan(NetArgs N, PlanPtrs P,
                                                                  uint32_t *netpre,
                                                                  uint32_t *netw) {
    __shared__ uint32_t lds[kNetBatch * kPlanWaves];
    __shared__ uint32_t pass[kMaxNetPasses][4];  // kind, k, lo, hi
    for (uint32_t p = threadIdx.x; p < N.np; p += kPlanThreads) {
        const uint32_t w = N.pass[p];
        pass[p][0] = w & 255u;
        pass[p][1] = (w >> 8) & 255u;
        pass[p][2] = (w >> 16) & 255u;
        pass[p][3] = w >> 24;
    }
    __syncthreads();
    const uint32_t n = P.work[W_SORT_TASKS];
    uint32_t a0, a1;
    owned_block(n, &a0, &a1);
    uint32_t bad = 0;
    for (uint32_t a = a0; a < a1; ++a) bad += (uint64_t)P.stab[a].m > (1ull << N.K);
    if (bad) atomicAdd(&P.work[W_ERRORS], 1u);
    for (uint32_t p0 = 0; p0 < N.np; p0 += kNetBatch) {
        const uint32_t nb = N.np - p0 < (uint32_t)kNetBatch ? N.np - p0 : (uint32_t)kNetBatch;
        uint32_t off[kNetBatch] = {}, tot[kNetBatch];
        for (uint32_t a = a0; a < a1; ++a) {
            const uint32_t m = P.stab[a].m;
#pragma unroll
            for (int i = 0; i < kNetBatch; ++i)
                if ((uint32_t)i < nb) {
                    const uint32_t *q = pass[p0 + i];
                    off[i] += bitonic_items_of(q[0], q[1], q[2], q[3], m, N.T);
                }
        }
        block_scan_n<kNetBatch, kPlanWaves>(off, tot, nb, lds);
        for (uint32_t a = a0; a < a1; ++a) {
            const uint32_t m = P.stab[a].m;
#pragma unroll
            for (int i = 0; i < kNetBatch; ++i)
                if ((uint32_t)i < nb) {
                    const uint32_t *q = pass[p0 + i];
                    netpre[(size_t)(p0 + i) * N.PS + a] = off[i];
                    off[i] += bitonic_items_of(q[0], q[1], q[2], q[3], m, N.T);
                }
        }
        if (threadIdx.x == 0)
            for (uint32_t i = 0; i < nb; ++i) netw[p0 + i] = tot[i];
    }
}

// ---- end of the schedule: segments still unsorted, plan errors -------------------
// status[0] accumulates errors, status[1] unsorted segments, until read.
__global__ __launch_bounds__(kBlock) void k_rounds_end(const DevSeg *seg, uint32_t nseg,
                                                       const uint32_t *work, uint32_t *status) {
    uint32_t left = 0;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < nseg; i += gridDim.x * kBlock)
        left += seg[i].flags != 0;
    if (left) atomicAdd(&status[1], left);
    if (blockIdx.x == 0 && threadIdx.x == 0 && work[W_ERRORS]) atomicAdd(&status[0], work[W_ERRORS]);
}

// Partition rounds per binary level between the longest segment and the
// loop's exit size (plus two): HybridQuickMergesort's rounds shrink a range
// with random keys to about 11/16 on average, 0.54 levels per round, and the
// network sorts what the slower ranges leave (on the 20,000-array batch 1.2,
// 1.5 and 2 rounds per level took 49.5, 49.9 and 50.7 ms with the first
// plan kernels, 46.7 and 46.9 ms with the present ones).
#ifndef QMS_DRC_ROUNDS_PER_LEVEL
#define QMS_DRC_ROUNDS_PER_LEVEL 1.2
#endif
constexpr double kRoundsPerLevel = QMS_DRC_ROUNDS_PER_LEVEL;

uint32_t ceil_log2_host(uint64_t x) {
    uint32_t l = 0;
    while ((1ull << l) < x) ++l;
    return l;
}

}  // namespace

// ---- host side ------------------------------------------------------------------
size_t rounds_state_bytes(uint32_t segs) {
    const size_t S = segs;
    return S * sizeof(DevSeg) + 3 * S * 4 + 2 * (S + 1) * sizeof(PartSeg) +
           (S + 1) * sizeof(SortSeg) + (9 + kMaxLevels) * (S + 2) * 4 + 64 * 4 +
           (size_t)kMaxNetPasses * (S + 2) * 4 + kMaxNetPasses * 4 +
           (size_t)(kPlanBlocks + 1) * kBlkStride * 4 + 16 * 256;
}

void carve_rounds_state(Workspace *ws, char *b, uint32_t segs) {
    const size_t S = segs;
    auto take = [&](size_t bytes) {
        char *p = b;
        b += (bytes + 255) & ~(size_t)255;
        return p;
    };
    ws->r_seg = take(S * sizeof(DevSeg));
    ws->r_aseg = (uint32_t *)take(S * 4);
    ws->r_live[0] = (uint32_t *)take(S * 4);
    ws->r_live[1] = (uint32_t *)take(S * 4);
    ws->r_ptab = take((S + 1) * sizeof(PartSeg));
    ws->r_mtab = take((S + 1) * sizeof(PartSeg));
    ws->r_stab = take((S + 1) * sizeof(SortSeg));
    ws->r_pre = (uint32_t *)take((9 + kMaxLevels) * (S + 2) * 4);
    ws->r_work = (uint32_t *)take(64 * 4);
    ws->r_status = (uint32_t *)take(4 * 4);
    ws->r_netpre = (uint32_t *)take((size_t)kMaxNetPasses * (S + 2) * 4);
    ws->r_netw = (uint32_t *)take(kMaxNetPasses * 4);
    ws->r_blk = (uint32_t *)take((size_t)(kPlanBlocks + 1) * kBlkStride * 4);
}

// The segments [h_off[j], h_off[j + 1]) of a batch, all below 2^32 keys;
// h_off: the host's copy of the offsets (for the schedule's bounds),
// d_offsets: the device's, or nullptr for a single array (h_off = {0, n}).
int sort_batch_device_rounds(int dt, bool pairs, char *keys_base, uint32_t *vals_base,
                             const uint64_t *d_offsets, const uint64_t *h_off, uint32_t nseg,
                             uint64_t loop_exit, Workspace &ws, hipStream_t st) {
    const Tuning tune = current_tuning();
    const bool wide = dtype_wide(dt);
    const uint32_t ew = wide ? 2 : 1;
    const uint32_t T0 = base_tile_of(pairs, wide);
    const bool auto_r0 = tune.base_tile == 0;
    // 64-bit keys with payloads merge two runs per pass
    const bool four_way = tune.merge_ways == 4 && !(pairs && wide);
    // automatic runs of kMergeTile keys for 64-bit keys and the logarithm
    // order (as the host-planned loop takes them), never halved
    const bool short_runs = wide || dt == QMS_U32_LOG;
    const uint32_t R0 = auto_r0 ? (short_runs ? (uint32_t)kMergeTile : T0) : std::min(T0, tune.base_tile);
    // the smallest run width a Mergesort can take (automatic: half of R0)
    const uint32_t R0_min = (auto_r0 && four_way && !short_runs) ? R0 / 2 : R0;
    const uint32_t S = ws.caps.segs;
    hipError_t e = hipSuccess;

    for (uint32_t g0 = 0; g0 < nseg;) {
        // a group: at most S segments and fewer than 2^32 keys
        uint32_t g1 = g0;
        uint64_t keys = 0, nmax = 0;
        while (g1 < nseg && g1 - g0 < S) {
            const uint64_t n = h_off[g1 + 1] - h_off[g1];
            if (g1 > g0 && keys + n >= (1ull << 32)) break;
            keys += n;
            nmax = std::max(nmax, n);
            ++g1;
        }
        const uint32_t G = g1 - g0;
        std::vector<uint64_t> len(G);
        for (uint32_t i = 0; i < G; ++i) len[i] = h_off[g0 + i + 1] - h_off[g0 + i];
        // the schedule: R partition rounds (every segment above the base
        // tile at least one), then the network on what is left
        const uint64_t F = std::max<uint64_t>(T0, std::min<uint64_t>(loop_exit, kMaxFinalTile));
        const double levels = nmax > F ? std::log2((double)nmax / F) : 0.0;
        const uint32_t R = nmax <= T0 ? 0
                           : nmax <= F ? 1
                                       : (uint32_t)std::ceil(kRoundsPerLevel * levels) + 2;
        // range bound of a segment of n keys after r rounds
        auto bound = [&](uint64_t n, uint32_t r) -> uint64_t {
            if (r <= 1) return n;
            const double b = (double)n * std::pow(15.0 / 16.0, (double)(r - 1)) + 72.0;
            return std::min<uint64_t>(n, (uint64_t)b);
        };
        // partition tile: the first round's tiles fit the workspace
        uint32_t TP = tune.partition_tile;
        for (;;) {
            uint64_t tot = 0;
            for (uint64_t n : len)
                if (n > T0) tot += (n + TP - 1) / TP;
            if (tot <= ws.caps.tiles) break;
            TP *= 2;
        }
        const uint32_t max_nt_all = (uint32_t)((nmax + TP - 1) / TP);
        const uint32_t scan_nth = max_nt_all > 4 * kBlock ? kScanThreads : kBlock;

        PlanArgs A{};
        A.nseg = G;
        A.TP = TP;
        A.scan_nth = scan_nth;
        A.span = tune.chunk_span;
        A.T0 = T0;
        A.R0 = R0;
        A.auto_r0 = auto_r0 && !short_runs;
        A.four_way = four_way;
        A.wide = wide;
        A.ew = ew;
        A.cap_tiles = (uint32_t)std::min<uint64_t>(ws.caps.tiles, 0xffffffffu);
        A.cap_chunks = (uint32_t)std::min<uint64_t>(ws.caps.chunks, 0xffffffffu);
        A.cap_splits = (uint32_t)std::min<uint64_t>(ws.caps.splits, 0xffffffffu);
        PlanPtrs P{};
        P.seg = (DevSeg *)ws.r_seg;
        P.aseg = ws.r_aseg;
        P.ptab = (PartSeg *)ws.r_ptab;
        P.mtab = (PartSeg *)ws.r_mtab;
        P.stab = (SortSeg *)ws.r_stab;
        const size_t PS = (size_t)G + 2;
        uint32_t *pre = ws.r_pre;
        P.p_tiles = pre;
        P.p_scan = pre + PS;
        P.p_mom = pre + 2 * PS;
        P.p_wa = pre + 3 * PS;
        P.p_ca = pre + 4 * PS;
        P.p_wb = pre + 5 * PS;
        P.p_cb = pre + 6 * PS;
        P.p_base = pre + 7 * PS;
        P.p_m2 = pre + 8 * PS;
        P.p_step = pre + 9 * PS;
        P.work = ws.r_work;
        P.meta = ws.meta;
        P.res = ws.res;

        hipLaunchKernelGGL(k_rounds_init, dim3(std::min<uint32_t>((G + kBlock - 1) / kBlock, 1024)),
                           dim3(kBlock), 0, st, P.seg, d_offsets, h_off[1], g0, G, (uint32_t *)keys_base,
                           vals_base, ew, T0, P.work);
        if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "round state init");

        // Launch sizes.  Each device-sized phase runs one workgroup per item
        // for as many items as the host expects (a median-of-3 round leaves
        // a range about 11/16 of its size on average; the estimate takes
        // 3/4 and a quarter more work), then a looping launch of kOverflow
        // workgroups for any items beyond the estimate (four per compute
        // unit, so that an estimate that falls short still runs on every
        // compute unit; 2,048 cost 0.3 ms more on the 20,000-array batch,
        // whose overflow launches are nearly all empty).  Where the host expects no
        // items, the looping launch alone is enqueued.  (One looping launch
        // per phase, sized from the estimate, was measured too: the looping
        // kernels run their items up to twice as slowly, and the batch took
        // 76 instead of 50 ms.)
#ifndef QMS_DRC_OVERFLOW
#define QMS_DRC_OVERFLOW 1024
#endif
        constexpr uint32_t kOverflow = QMS_DRC_OVERFLOW;
        constexpr double kShrink = 0.75, kSlack = 1.25;
        auto est = [](double x) -> uint32_t {
            if (x <= 0.0) return 0;
            return (uint32_t)std::min<double>(std::ceil(x * kSlack) + 16.0, 1u << 30);
        };
        // device-sized task references: the work-item count and the number
        // of segments in the table are read from the plan's counters
        auto part_ref = [&](const uint32_t *prefix, uint32_t work_slot, const PartSeg *tab,
                            uint32_t count_slot = W_ACTIVE) {
            TaskRef<PartSeg> r{};
            r.tab = tab;
            r.pre = prefix;
            r.A = G + 1;  // an upper bound (>= 2: never the by-value form)
            r.dyn = P.work + work_slot;
            r.dyn_A = P.work + count_slot;
            return r;
        };
        auto sort_ref = [&](const uint32_t *prefix, uint32_t work_slot) {
            TaskRef<SortSeg> r{};
            r.tab = P.stab;
            r.pre = prefix;
            r.A = G + 1;
            r.dyn = P.work + work_slot;
            r.dyn_A = P.work + W_SORT_TASKS;
            return r;
        };

        const uint32_t NBp = (G + kPB - 1) / kPB;  // plan workgroups
        std::vector<double> expect(G);  // expected range of each segment
        std::vector<char> was_act(G, 0);  // partitioned in the previous round
        for (uint32_t i = 0; i < G; ++i) expect[i] = (double)len[i];
        for (uint32_t r = 0; r <= R; ++r) {
            // live lists: every segment in the first round, then the list the
            // previous round's side kernel compacted
            P.live_in = r == 0 ? nullptr : ws.r_live[(r - 1) & 1];
            P.live_out = ws.r_live[r & 1];
            // estimates of this round's work, and the bound on the largest
            // range (for the number of merge steps, which must not fall short)
            double tiles_e = 0, scan_e = 0, chunks_e = 0, active_e = 0, mom_e = 0, merge_e = 0;
            double base_e = 0;
            uint64_t bmax = 0, tiles_b = 0;
            for (uint32_t i = 0; i < G; ++i) {
                const uint64_t n = len[i];
                if (n <= 1) continue;
                const double x = expect[i];
                const uint64_t b = bound(n, r);
                if (r < R && b > T0) {
                    bmax = std::max(bmax, b);
                    tiles_b += (b + TP - 1) / TP;
                }
                // partitioned this round: every segment above the base tile
                // in the first round, then the ranges above the loop's exit
                const bool act = r < R && (r == 0 ? x > T0 : x > (double)F);
                if (act) {
                    const double nt = std::ceil(x / TP);
                    tiles_e += nt;
                    scan_e += scan_a_groups((uint32_t)nt, scan_nth);
                    // exchange chunks: about s / span, or X / kRankChunk when
                    // the X misplaced pairs (about s / 4 for keys in random
                    // order) fill the chunks first
                    chunks_e += std::ceil(std::max(x / std::max<uint32_t>(tune.chunk_span, 4096),
                                                   x / 4 / kRankChunk)) + 1;
                    active_e += 1;
                    mom_e += 0.1 * mom_tiles((uint64_t)x);
                    merge_e += std::ceil(0.35 * x / kMergeTile);
                    base_e += std::ceil(0.35 * x / T0);
                }
                // the ranges that reach the base tile: base case next round;
                // the last round: the tiles of the ranges the network finishes
                if (x <= T0 && (r == 0 || was_act[i])) base_e += 1;
                if (r == R && x > T0) base_e += std::ceil(x / T0);
                was_act[i] = act;
                if (act) expect[i] = x * kShrink;
            }
            const uint32_t Lmax = bmax / 2 > R0_min ? ceil_log2_host((bmax / 2 + R0_min - 1) / R0_min) : 0;
            const uint32_t steps = std::min<uint32_t>(four_way ? Lmax / 2 : Lmax, kMaxLevels);
            A.F = (uint32_t)F;
            A.xfinal = r == R ? 1u : 0u;
            A.steps = steps;
            A.first2 = four_way && (!auto_r0 || short_runs) && Lmax > 0;
            A.partitioned = r < R && bmax > 0;
            if (A.partitioned) {
                hipLaunchKernelGGL(k_rounds_plan_count, dim3(NBp), dim3(kPB), 0, st, A, P, ws.r_blk);
                hipLaunchKernelGGL(k_rounds_plan_write, dim3(NBp), dim3(kPB), 0, st, A, P,
                                   (const uint32_t *)ws.r_blk);
                // pivots of the flagged ranges: the estimated launch always
                // takes the first items (a looping launch that also took the
                // first items gave wrong pivots on a batch of 409 arrays;
                // the cause is not known)
                e = launch_mom_pivot(dt, part_ref(P.p_mom, W_MOM, P.mtab, W_MOM_SEGS),
                                     std::max<uint32_t>(est(mom_e), 16), kOverflow,
                                     false, ws, st);
                if (e != hipSuccess) return hip_error(e, "median-of-medians pivot");
                PartitionLaunch L{};
                L.TP = TP;
                L.chunk_span = tune.chunk_span;
                L.scan_threads = scan_nth;
                // per-64 counts while the round's tiles (at most tiles_b) fit
                L.groups = tiles_b * (TP / kWave) <= ws.caps.groups;
                L.keys_total = 0;
                L.bytes = 0;
                L.ws = &ws;
                L.work = 0;
                // the phase with an estimate of `items` workgroups, then the
                // overflow from where the estimate ends (items per workgroup:
                // one, or kWaves for the splits)
                auto phase = [&](int ph, TaskRef<PartSeg> tr, uint32_t items, uint32_t per,
                                 const char *what) -> int {
                    L.phase = ph;
                    L.tasks = tr;
                    L.grid = (items + per - 1) / per;
                    L.first = 0;
                    L.loop = false;
                    hipError_t e2 = launch_partition_phase(dt, pairs, L, st);
                    if (e2 == hipSuccess) {
                        L.first = L.grid * per;
                        L.grid = kOverflow;
                        L.loop = true;
                        e2 = launch_partition_phase(dt, pairs, L, st);
                    }
                    return e2 == hipSuccess ? QMS_OK : hip_error(e2, what);
                };
                int rc;
                if ((rc = phase(0, part_ref(P.p_tiles, W_TILES, P.ptab), est(tiles_e), 1,
                                "partition count")) != QMS_OK)
                    return rc;
                if ((rc = phase(6, part_ref(P.p_scan, W_SCAN, P.ptab), est(scan_e), 1,
                                "partition scan")) != QMS_OK)
                    return rc;
                hipLaunchKernelGGL(k_rounds_swap_count, dim3(NBp), dim3(kPB), 0, st, A, P, ws.r_blk);
                hipLaunchKernelGGL(k_rounds_swap_write, dim3(NBp), dim3(kPB), 0, st, A, P,
                                   (const uint32_t *)ws.r_blk);
                if ((rc = phase(1, part_ref(P.p_wa, W_SPLIT_A, P.ptab), est(2 * chunks_e), kWaves,
                                "split A")) != QMS_OK)
                    return rc;
                if ((rc = phase(2, part_ref(P.p_ca, W_SWAP_A, P.ptab), est(chunks_e), 1,
                                "swap A")) != QMS_OK)
                    return rc;
                if ((rc = phase(4, part_ref(nullptr, W_ACTIVE, P.ptab), est(active_e), 1,
                                "scan B")) != QMS_OK)
                    return rc;
                if ((rc = phase(3, part_ref(P.p_wb, W_SPLIT_B, P.ptab), 16, kWaves, "split B")) !=
                    QMS_OK)
                    return rc;
                if ((rc = phase(5, part_ref(P.p_cb, W_SWAP_B, P.ptab), 16, 1, "swap B")) != QMS_OK)
                    return rc;
            }
            // side choice (or, after the last round, the finals alone)
            hipLaunchKernelGGL(k_rounds_side_count, dim3(NBp), dim3(kPB), 0, st, A, P, ws.r_blk);
            hipLaunchKernelGGL(k_rounds_side_write, dim3(NBp), dim3(kPB), 0, st, A, P,
                               (const uint32_t *)ws.r_blk);
            e = launch_tile_sort(dt, pairs, sort_ref(P.p_base, W_BASE), est(base_e), kOverflow, 0.0,
                                 ws, st);
            if (e != hipSuccess) return hip_error(e, "base case");
            if (steps == 0 && !A.first2) continue;
            MergeLaunch M;
            M.overflow = kOverflow;
            M.tiles = est(merge_e);
            // the 2-way first passes of odd level counts (never with the
            // automatic run width, which makes every level count even)
            if (A.first2) {
                M.tasks = sort_ref(P.p_m2, W_MERGE2);
                M.level = 0;
                M.step = 0;
                M.four_way = false;
                if ((e = launch_merge_pass(dt, pairs, M, ws, st)) != hipSuccess)
                    return hip_error(e, "merge pass");
            }
            for (uint32_t k = 0; k < steps; ++k) {
                M.tasks = sort_ref(P.p_step + (size_t)k * PS, W_STEP0 + k);
                M.level = k;
                M.step = 1;
                M.four_way = four_way;
                if ((e = launch_merge_pass(dt, pairs, M, ws, st)) != hipSuccess)
                    return hip_error(e, "merge pass");
            }
        }
        // X at the loop level: the network on every range the last round
        // handed over (their tiles sorted in place by that round's base
        // case), enqueued for the largest range the schedule's bound allows
        const uint64_t fmax = R == 0 ? 0 : std::min<uint64_t>(nmax, std::max<uint64_t>(F, bound(nmax, R)));
        const uint32_t lt = ceil_log2_host(T0);
        const uint32_t Kn = fmax > T0 ? ceil_log2_host(fmax) : 0;
        if (Kn > lt) {
            const std::vector<BitonicLaunch> passes = bitonic_passes(Kn, lt);
            if (passes.size() > kMaxNetPasses)
                return set_error(QMS_ERR_UNSUPPORTED, "network plan beyond its table");
            NetArgs N{};
            N.K = Kn;
            N.T = T0;
            N.np = (uint32_t)passes.size();
            N.PS = (uint32_t)PS;
            for (size_t p = 0; p < passes.size(); ++p)
                N.pass[p] = passes[p].kind | passes[p].k << 8 | passes[p].lo << 16 | passes[p].hi << 24;
            hipLaunchKernelGGL(k_rounds_net_plan, dim3(1), dim3(kPlanThreads), 0, st, N, P,
                               ws.r_netpre, ws.r_netw);
            if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "network plan");
            for (size_t p = 0; p < passes.size(); ++p) {
                BitonicLaunch L = passes[p];
                L.tasks.tab = P.stab;
                L.tasks.pre = ws.r_netpre + p * PS;
                L.tasks.A = G + 1;
                L.tasks.dyn = ws.r_netw + p;
                L.tasks.dyn_A = P.work + W_SORT_TASKS;
                L.items = kOverflow;
                if ((e = launch_bitonic_pass(dt, pairs, L, st)) != hipSuccess)
                    return hip_error(e, "bitonic network");
            }
        }
        hipLaunchKernelGGL(k_rounds_end, dim3(std::min<uint32_t>((G + kBlock - 1) / kBlock, 1024)),
                           dim3(kBlock), 0, st, (const DevSeg *)P.seg, G,
                           (const uint32_t *)P.work, ws.r_status);
        if ((e = hipGetLastError()) != hipSuccess) return hip_error(e, "round schedule end");
        g0 = g1;
    }
    return QMS_OK;
}

}  // namespace qms
