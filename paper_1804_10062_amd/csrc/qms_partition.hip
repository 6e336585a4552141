// qms_partition.hip -- in-place three-way partition around a median-of-3
// pivot on gfx950.
//
// The paper leaves the partition routine open (Sec. "QuickMergeXsort": "the
// partitioning algorithm [has] to be added"); its pivot is the median of a
// sample of three (Theorem 1), and Sec. "Worst-Case Efficient QuickMergeSort"
// notes that with duplicate keys the elements equal to the pivot should go
// to the middle and take part in neither Mergesort nor the recursion.  This
// file implements exactly that partition of a range [lo, hi):
//
//     [lo, B1) < p      [B1, B2) == p      [B2, hi) > p
//
// in place, in two passes of the same rank-matched exchange:
//   pass A  splits "< p" from ">= p" at B1 = lo + #(< p);
//   pass B  splits "== p" from "> p" inside [B1, hi) at B2 = B1 + #(== p).
// A pass pairs the k-th misplaced element of the left region with the k-th
// misplaced element of the right region and exchanges them; the pairing is a
// perfect matching, so every element moves at most once per pass.
//
// Kernels, per pass:
//   count   one workgroup per tile: #(< p) and #(== p) of the tile, and
//           #(< p) of every 64 positions (pass A);
//   scan    up to kScanGroups workgroups per segment: totals, boundary,
//           per-tile misplaced counts and their exclusive prefix sums (ranks
//           of each tile's first misplaced element on either side), and for
//           every chunk boundary (rank j * rc) the tile that holds it;
//   split   one wave per chunk boundary and side: the exact position of the
//           misplaced element of rank j * rc inside that tile (from the
//           per-64 counts and one ballot, or by walking the tile);
//   swap    one workgroup per chunk: reads exactly the position ranges of its
//           ranks on both sides (coalesced, wave-striped), compacts the
//           misplaced elements with ballot + prefix counts into LDS, and
//           writes them exchanged.
// Chunks own disjoint position ranges, so no workgroup reads a cell another
// one writes.  Pass B's per-tile counts are derived from pass A's without a
// second counting sweep: equal keys in the right region never move in pass A,
// and pass A counts (atomically, per tile) the equal keys it moves in.
//
// All kernels serve every segment of a round at once (task tables, see
// qms_device.hpp).  Workspace: per-tile counters and per-chunk boundaries of
// fixed capacity; positions are 32-bit offsets from the segment base.
#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

namespace qms {

__device__ __forceinline__ const PartSeg &seg_by_index(const TaskRef<PartSeg> &r, uint32_t a) {
    return r.A == 1 ? r.one : r.tab[a];
}

// ---- count -------------------------------------------------------------------
// One workgroup per tile: #(< p) and #(== p).  With `gcnt`, also #(< p) in
// each 64 positions of the tile (one wave's ballot; a byte per group, TP / 64
// per tile), from which the split finds a chunk boundary's 64 positions
// without walking the tile.
template <class O>
__device__ __forceinline__ void part_count_item(TaskRef<PartSeg> tasks, uint32_t item,
                                                uint32_t TP, uint32_t *cnt_lt, uint32_t *cnt_eq,
                                                uint8_t *gcnt, const uint64_t *meta,
                                                uint32_t *tmp) {
    using K = typename O::K;
    uint32_t t, a;
    const PartSeg g = task_of(tasks, item, &t, &a);
    const K *keys = (const K *)g.keys + g.lo;
    const uint64_t ts = (uint64_t)t * TP;
    const uint64_t te = ts + TP < g.s ? ts + TP : g.s;
    uint32_t lt = 0, eq = 0;
    K p = 0;
    for (uint64_t b = ts; b < te; b += kPartSub) {
        // clamped, unconditional loads (all in flight together); the tail
        // positions are masked out of the counts
        K k[kPartItems];
#pragma unroll
        for (int q = 0; q < kPartItems; ++q) {
            const uint64_t pos = b + (uint64_t)q * kBlock + threadIdx.x;
            k[q] = ldg(keys + (pos < te ? pos : te - 1));
        }
        // the pivot's loads go out behind the tile's (before them, their wait
        // held the tile's loads back: two memory latencies per workgroup)
        if (b == ts)
            p = (g.flags & kPivotMoM) ? (K)ldg(meta + (uint64_t)g.slot * M_COUNT + M_PIVOT)
                                      : pivot_of<O>(keys, 0, g.s);
        uint32_t mine = 0;  // lane q: this wave's count in slice q
#pragma unroll
        for (int q = 0; q < kPartItems; ++q) {
            const uint64_t pos = b + (uint64_t)q * kBlock + threadIdx.x;
            const K x = O::ord(k[q]);
            const bool in = pos < te;
            const bool less = in && O::lt(x, p);
            lt += less;
            eq += in && x == p;
            if (gcnt) {
                const uint32_t c = (uint32_t)__popcll(__ballot(less));
                mine = lane_id() == q ? c : mine;
            }
        }
        if (gcnt && lane_id() < kPartItems) {
            // the wave's 64 positions of slice `lane`
            const uint64_t g0 = b + (uint64_t)lane_id() * kBlock + (uint64_t)wave_id() * kWave;
            if (g0 < te)
                gcnt[((uint64_t)g.tile_off + t) * (TP / kWave) + (g0 - ts) / kWave] = (uint8_t)mine;
        }
    }
    lt = block_sum(lt, tmp);
    eq = block_sum(eq, tmp);  // ends with a barrier: tmp is free again
    if (threadIdx.x == 0) {
        cnt_lt[g.tile_off + t] = lt;
        cnt_eq[g.tile_off + t] = eq;
    }
}
template <class O, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_part_count(TaskRef<PartSeg> tasks, uint32_t first,
                                                       uint32_t TP, uint32_t *cnt_lt,
                                                       uint32_t *cnt_eq, uint8_t *gcnt,
                                                       const uint64_t *meta) {
    __shared__ uint32_t tmp_lds[kWaves + 1];
    uint32_t *tmp = tmp_lds;
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) part_count_item<O>(tasks, item, TP, cnt_lt, cnt_eq, gcnt, meta, tmp);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            part_count_item<O>(tasks, item, TP, cnt_lt, cnt_eq, gcnt, meta, tmp);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}

// count keys with ord(k) < p and == p in [a, b) (a < b) with the whole
// block, four clamped loads per thread in flight
template <class O>
__device__ __forceinline__ void block_count_range(const typename O::K *keys, uint64_t a,
                                                  uint64_t b, typename O::K p, uint32_t *lt_out,
                                                  uint32_t *eq_out, uint32_t *tmp) {
    using K = typename O::K;
    uint32_t lt = 0, eq = 0;
    const uint64_t nth = blockDim.x;
    for (uint64_t base = a; base < b; base += 4 * nth) {
        K k[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t pos = base + q * nth + threadIdx.x;
            k[q] = ldg(keys + (pos < b ? pos : b - 1));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t pos = base + q * nth + threadIdx.x;
            const K x = O::ord(k[q]);
            lt += pos < b && O::lt(x, p);
            eq += pos < b && x == p;
        }
    }
    *lt_out = block_sum(lt, tmp);
    *eq_out = block_sum(eq, tmp);
}

// Exclusive prefix sums of the per-tile misplaced counts of both sides.  The
// per-tile words are staged through LDS in chunks of NTH * kScanPer tiles
// (coalesced loads, all in flight); each thread then scans kScanPer
// consecutive tiles of the chunk.  ld(t) gives tile t's words, mis(t, w, &l,
// &r) its counts from them.  Returns the left side's total.
template <int NTH>
struct ScanStage {
    uint2 w[NTH * kScanPer + NTH];  // one spare slot every kScanPer (bank spread)
};
template <int NTH, class LD, class MIS>
__device__ __forceinline__ uint32_t scan_misplaced(uint32_t nt, LD ld, MIS mis, uint32_t *preL,
                                                   uint32_t *preR, ScanStage<NTH> &stage,
                                                   uint32_t *tmp) {
    constexpr uint32_t C = (uint32_t)NTH * kScanPer;
    const uint32_t tid = threadIdx.x;
    uint32_t carryL = 0, carryR = 0;
    for (uint32_t c0 = 0; c0 < nt; c0 += C) {
        uint2 v[kScanPer];
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const uint32_t t = c0 + (uint32_t)q * NTH + tid;
            v[q] = ld(t < nt ? t : nt - 1);
        }
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const uint32_t e = (uint32_t)q * NTH + tid;
            stage.w[e + e / kScanPer] = v[q];
        }
        __syncthreads();
        uint32_t l[kScanPer], r[kScanPer], sl = 0, sr = 0;
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) {
            const uint32_t e = tid * kScanPer + (uint32_t)i;
            l[i] = r[i] = 0;
            if (c0 + e < nt) mis(c0 + e, stage.w[e + e / kScanPer], &l[i], &r[i]);
            sl += l[i];
            sr += r[i];
        }
        // the scans end with a barrier, after which the stage may be refilled
        uint32_t totL, totR;
        uint32_t offL = carryL + block_exclusive_scan(sl, tmp, &totL);
        uint32_t offR = carryR + block_exclusive_scan(sr, tmp, &totR);
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) {
            const uint32_t t = c0 + tid * kScanPer + (uint32_t)i;
            if (t < nt) {
                stg(preL + t, offL);
                stg(preR + t, offR);
            }
            offL += l[i];
            offR += r[i];
        }
        carryL += totL;
        carryR += totR;
    }
    if (tid == 0) {
        stg(preL + nt, carryL);
        stg(preR + nt, carryR);
    }
    return carryL;
}

// Chunk boundaries j = 1 .. nch - 1 lie at the misplaced elements of rank
// j * rc of each side.  For every tile, record for each boundary whose rank
// falls in the tile the tile and the boundary's rank inside it, encoded as
// t * TP + k (< the range size); k_part_split turns it into a position.
// mark_boundaries does it for the ranks [a, b) of tile t on one side (a
// 32-bit division: a 64-bit one cost the one-workgroup scans a hundred
// instructions per tile).
__device__ __forceinline__ void mark_boundaries(uint32_t *sp, uint32_t a, uint32_t b, uint32_t t,
                                                uint32_t TP, uint32_t rc, uint32_t nch) {
    uint32_t j = a / rc;
    if ((uint64_t)j * rc < a) ++j;
    if (j == 0) j = 1;
    for (; j < nch && (uint64_t)j * rc < b; ++j)
        stg(sp + j, (uint32_t)((uint64_t)t * TP + ((uint64_t)j * rc - a)));
}
// The same for every tile of pass B, from the prefixes the block has just
// written.
template <int NTH>
__device__ __forceinline__ void mark_chunk_tiles(uint32_t nt, uint32_t TP, uint32_t rc,
                                                 uint32_t nch, const uint32_t *preL,
                                                 const uint32_t *preR, uint32_t *spL,
                                                 uint32_t *spR) {
    __syncthreads();  // prefixes written by other threads of the block
    if (nch <= 1) return;
    constexpr uint32_t C = (uint32_t)NTH * 4;
    for (uint32_t c0 = 0; c0 < nt; c0 += C) {
        uint32_t l0[4], l1[4], r0[4], r1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t t = c0 + (uint32_t)q * NTH + threadIdx.x;
            t = t < nt ? t : nt - 1;
            l0[q] = ldg(preL + t);
            l1[q] = ldg(preL + t + 1);
            r0[q] = ldg(preR + t);
            r1[q] = ldg(preR + t + 1);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t t = c0 + (uint32_t)q * NTH + threadIdx.x;
            if (t < nt) {
                if (l1[q] > l0[q]) mark_boundaries(spL, l0[q], l1[q], t, TP, rc, nch);
                if (r1[q] > r0[q]) mark_boundaries(spR, r0[q], r1[q], t, TP, rc, nch);
            }
        }
    }
}

// ---- scan of pass A ----------------------------------------------------------
// The tiles of a segment are cut into chunks of C = NTH * kScanPer; up to
// kScanGroups workgroups serve the segment, each owning a run of
// consecutive chunks.  Every workgroup
//   1. sums the counts of all tiles (loads and adds only: with no stores in
//      the loop, the next chunk's loads stay in flight while a chunk is
//      added up): #(< p) per chunk, whose exclusive prefix is each chunk's
//      carry, and the totals c_lt and c_eq;
//   2. with B1 = c_lt in tile tb, lt_part = #(< p) in [tb TP, B1) and
//      P[t] = #(< p) in tiles before t, every tile left of tb is full and
//      wholly left of B1, so the misplaced ranks have closed forms:
//        preL[t] = t TP - P[t]                (t <= tb),  X  (t > tb)
//        preR[t] = 0                          (t <= tb),  P[t] - P[tb] - lt_part  (t > tb)
//      with X = c_lt - P[tb] - lt_part pairs.  For its own chunks it writes
//      them, records the tile of every chunk boundary and clears eqmv.
// Workgroup 0 writes the round state and res[4 a + 0..2] = (#<p, #==p,
// pass-A pairs) for the host.  (One workgroup walking all chunks in turn
// waited at each chunk for the previous chunk's stores to drain, since a
// load's wait also covers the stores issued before it: about 5 us per
// 8,192 tiles on the largest ranges.)
// Work items: the task prefix counts each segment's workgroups
// (min(chunks of tiles, kScanGroups)); item -> (segment a, group kgrp).
template <int NTH>
struct ScanALds {
    static constexpr uint32_t C = (uint32_t)NTH * kScanPer;
    static constexpr uint32_t kMaxChunks = (uint32_t)(kCapTiles / C) + 1;
    uint32_t tmp[NTH / kWave + 1];
    uint32_t csum[kMaxChunks];  // #(< p) per chunk, then its carry
    uint32_t stage[C + NTH + 1];  // one spare slot every kScanPer (bank spread)
};
template <class O, int NTH>
__device__ __forceinline__ void part_scan_a_item(TaskRef<PartSeg> tasks, uint32_t item,
                                                 uint32_t TP, uint32_t span,
                                                 const uint32_t *cnt_lt_all,
                                                 const uint32_t *cnt_eq_all, uint32_t *preL_all,
                                                 uint32_t *preR_all, uint32_t *eqmv_all,
                                                 uint32_t *spL_all, uint32_t *spR_all,
                                                 uint64_t *meta_all, uint32_t *res,
                                                 ScanALds<NTH> &lds) {
    constexpr int PER = kScanPer;
    constexpr uint32_t C = (uint32_t)NTH * PER;
    static_assert(kCapTiles / ((uint64_t)kScanThreads * kScanPer) < kScanThreads,
                  "one thread per chunk carries the chunks' prefix");
    uint32_t *tmp = lds.tmp, *csum = lds.csum, *stage = lds.stage;
    using K = typename O::K;
    uint32_t kgrp, a;
    const PartSeg g = task_of_wave(tasks, item, &kgrp, &a);
    const K *keys = (const K *)g.keys + g.lo;
    const uint32_t *LT = cnt_lt_all + g.tile_off;
    const uint32_t *EQ = cnt_eq_all + g.tile_off;
    uint32_t *preL = preL_all + g.tile_off + g.slot;
    uint32_t *preR = preR_all + g.tile_off + g.slot;
    uint32_t *eqmv = eqmv_all + g.tile_off;
    uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
    const uint32_t nt = g.nt;
    const uint64_t s = g.s;
    const uint32_t tid = threadIdx.x;
    const uint32_t nch_t = (nt + C - 1) / C;  // chunks of tiles
    const uint32_t G = scan_a_groups(nt, NTH);
    if (kgrp >= G) return;
    const uint32_t k0 = (uint32_t)((uint64_t)kgrp * nch_t / G);
    const uint32_t k1 = (uint32_t)((uint64_t)(kgrp + 1) * nch_t / G);
    for (uint32_t k = tid; k < nch_t; k += NTH) csum[k] = 0;
    const K p = (g.flags & kPivotMoM) ? (K)ldg(meta + M_PIVOT) : pivot_of<O>(keys, 0, s);
    __syncthreads();
    // pass 1
    auto load_counts = [&](uint32_t c0, uint2(&v)[PER]) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t t = c0 + (uint32_t)q * NTH + tid;
            v[q] = t < nt ? make_uint2(ldg(LT + t), ldg(EQ + t)) : make_uint2(0u, 0u);
        }
    };
    uint32_t seq = 0;
    {
        uint2 v[PER];
        load_counts(0, v);
        for (uint32_t k = 0; k < nch_t; ++k) {
            uint32_t sl = 0;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                sl += v[q].x;
                seq += v[q].y;
            }
            if (k + 1 < nch_t) load_counts((k + 1) * C, v);
            sl = wave_inclusive_scan(sl);
            if (lane_id() == kWave - 1) atomicAdd(&csum[k], sl);
        }
    }
    __syncthreads();
    uint64_t c_lt;
    {
        const uint32_t mine = tid < nch_t ? csum[tid] : 0u;
        uint32_t tot;
        const uint32_t carry = block_exclusive_scan(mine, tmp, &tot);  // ends with a barrier
        if (tid < nch_t) csum[tid] = carry;
        c_lt = tot;
    }
    const uint64_t c_eq_all = block_sum(seq, tmp);  // (its barriers publish csum)
    // Keys equal to the pivot get a block of their own (pass B) only when
    // there are many of them, or when nothing is smaller than the pivot (then
    // excluding them is what makes the round progress).  Otherwise they stay
    // in the ">= p" side, where the sort treats them like any other key; the
    // round still removes at least one key from the range (the "< p" side).
    const bool eq_block = c_lt == 0 || c_eq_all > kEqBlockMin + s / 4096;
    const uint64_t c_eq = eq_block ? c_eq_all : 0;
    const uint32_t tb = (uint32_t)(c_lt / TP);  // tile holding B1 (tb < nt since c_lt < s)
    uint32_t lt_part = 0, eq_part = 0;
    if (c_lt % TP != 0) block_count_range<O>(keys, (uint64_t)tb * TP, c_lt, p, &lt_part, &eq_part, tmp);
    // P[tb]: the carry of tb's chunk and the tiles before tb in it
    uint32_t Ptb;
    {
        const uint32_t kb = tb / C;
        uint32_t part = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t t = kb * C + (uint32_t)q * NTH + tid;
            part += t < tb ? ldg(LT + t) : 0u;
        }
        Ptb = csum[kb] + block_sum(part, tmp);
    }
    const uint32_t X = (uint32_t)c_lt - Ptb - lt_part;
    const uint32_t rc = rank_chunk(X, s, span);
    const uint32_t nch = (uint32_t)chunk_count(X, s, span);
    uint32_t *spL = spL_all + g.chunk_off, *spR = spR_all + g.chunk_off;
    // pass 2, over this workgroup's chunks
    auto prefix_at = [&](uint32_t t, uint32_t Pt, uint32_t *l, uint32_t *r) {
        *l = t <= tb ? t * TP - Pt : X;
        *r = t <= tb ? 0u : Pt - Ptb - lt_part;
    };
    for (uint32_t k = k0; k < k1; ++k) {
        const uint32_t c0 = k * C;
        // #(< p) per tile, coalesced, into LDS; each thread then takes PER
        // consecutive tiles, and the block scan turns them into P
        uint32_t v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t t = c0 + (uint32_t)q * NTH + tid;
            v[q] = t < nt ? ldg(LT + t) : 0u;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)q * NTH + tid;
            stage[e + e / PER] = v[q];
        }
        __syncthreads();
        uint32_t mine[PER], sl = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t e = tid * PER + (uint32_t)i;
            mine[i] = stage[e + e / PER];
            sl += mine[i];
        }
        uint32_t tot;
        uint32_t off = csum[k] + block_exclusive_scan(sl, tmp, &tot);  // ends with a barrier
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t e = tid * PER + (uint32_t)i;
            stage[e + e / PER] = off;  // P[c0 + e]
            off += mine[i];
        }
        if (tid == NTH - 1) stage[C + C / PER] = off;  // P at the chunk's end
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const uint32_t e = (uint32_t)q * NTH + tid;
            const uint32_t t = c0 + e;
            if (t < nt) {
                // P[nt] = c_lt: tiles past nt count zero
                const uint32_t Pt = stage[e + e / PER], Pt1 = stage[e + 1 + (e + 1) / PER];
                uint32_t l0, r0, l1, r1;
                prefix_at(t, Pt, &l0, &r0);
                prefix_at(t + 1, Pt1, &l1, &r1);
                stg(preL + t, l0);
                stg(preR + t, r0);
                stg(eqmv + t, 0u);
                if (t == nt - 1) {
                    stg(preL + nt, l1);
                    stg(preR + nt, r1);
                }
                if (nch > 1) {
                    // left of tb only left ranks, right of it only right ones
                    const bool right = t > tb;
                    const uint32_t ra = right ? r0 : l0, rb = right ? r1 : l1;
                    if (rb > ra) mark_boundaries(right ? spR : spL, ra, rb, t, TP, rc, nch);
                    if (t == tb && r1 > r0) mark_boundaries(spR, r0, r1, t, TP, rc, nch);
                }
            }
        }
        __syncthreads();  // the stage is reused by the next chunk
    }
    if (kgrp == 0 && tid == 0) {
        meta[M_RCA] = rc;
        meta[M_PIVOT] = p;
        meta[M_CLT] = c_lt;
        meta[M_CEQ] = c_eq;
        meta[M_XA] = X;
        meta[M_TB] = tb;
        meta[M_LTPART] = lt_part;
        meta[M_EQPART] = eq_part;
        meta[M_XB] = 0;
        spL[0] = 0;
        spL[nch] = (uint32_t)c_lt;
        spR[0] = (uint32_t)c_lt;
        spR[nch] = (uint32_t)s;
        res[4 * a + 0] = (uint32_t)c_lt;
        res[4 * a + 1] = (uint32_t)c_eq;
        res[4 * a + 2] = X;
        res[4 * a + 3] = 0;
    }
}
template <class O, int NTH, bool LOOP>
__global__ __launch_bounds__(NTH) void k_part_scan_a(TaskRef<PartSeg> tasks, uint32_t first,
                                                     uint32_t TP, uint32_t span,
                                                     const uint32_t *cnt_lt_all,
                                                     const uint32_t *cnt_eq_all,
                                                     uint32_t *preL_all, uint32_t *preR_all,
                                                     uint32_t *eqmv_all, uint32_t *spL_all,
                                                     uint32_t *spR_all, uint64_t *meta_all,
                                                     uint32_t *res) {
    __shared__ ScanALds<NTH> lds_mem;
    ScanALds<NTH> *lds = &lds_mem;
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) part_scan_a_item<O, NTH>(tasks, item, TP, span, cnt_lt_all, cnt_eq_all, preL_all,
                                     preR_all, eqmv_all, spL_all, spR_all, meta_all, res, *lds);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            part_scan_a_item<O, NTH>(tasks, item, TP, span, cnt_lt_all, cnt_eq_all, preL_all,
                                     preR_all, eqmv_all, spL_all, spR_all, meta_all, res, *lds);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}

// ---- scan of pass B ----------------------------------------------------------
// After pass A, [B1, s) holds only keys >= p.  The keys == p of a tile's part
// right of B1 are the ones it held before (they did not move) plus the ones
// pass A moved in (eqmv).  One workgroup per segment; segments without
// possible pass-B pairs return at once.
template <int NTH>
struct ScanBLds {
    uint32_t tmp[NTH / kWave + 1];
    ScanStage<NTH> stage;
};
template <class O, int NTH>
__device__ __forceinline__ void part_scan_b_item(TaskRef<PartSeg> tasks, uint32_t item,
                                                 uint32_t TP, uint32_t span,
                                                 const uint32_t *cnt_eq_all,
                                                 const uint32_t *eqmv_all, uint32_t *preL_all,
                                                 uint32_t *preR_all, uint32_t *spL_all,
                                                 uint32_t *spR_all, uint64_t *meta_all,
                                                 ScanBLds<NTH> &lds) {
    uint32_t *tmp = lds.tmp;
    ScanStage<NTH> &stage = lds.stage;
    const PartSeg g = seg_by_index(tasks, item);
    uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
    const uint64_t s = g.s;
    const uint64_t b1 = meta[M_CLT];
    const uint64_t b2 = b1 + meta[M_CEQ];
    if (b2 >= s || b2 == b1) {
        if (threadIdx.x == 0) meta[M_XB] = 0;
        return;
    }
    using K = typename O::K;
    const K *keys = (const K *)g.keys + g.lo;
    const uint32_t *cnt_eq = cnt_eq_all + g.tile_off;
    const uint32_t *eqmv = eqmv_all + g.tile_off;
    uint32_t *preL = preL_all + g.tile_off + g.slot;
    uint32_t *preR = preR_all + g.tile_off + g.slot;
    const uint32_t nt = g.nt;
    const K p = (K)meta[M_PIVOT];
    const uint64_t tb = meta[M_TB];
    const uint32_t eq_part = (uint32_t)meta[M_EQPART];
    const uint64_t tb2 = b2 / TP;
    uint32_t eq_part2 = 0, dummy = 0;
    if (b2 % TP != 0 && tb2 < nt) {
        const uint64_t a = tb2 * TP > b1 ? tb2 * TP : b1;
        block_count_range<O>(keys, a, b2, p, &dummy, &eq_part2, tmp);
    }
    auto ld = [&](uint32_t t) { return make_uint2(ldg(cnt_eq + t), ldg(eqmv + t)); };
    auto mis = [&](uint32_t t, uint2 w, uint32_t *l, uint32_t *r) {
        if (t < tb) {
            *l = 0;
            *r = 0;
            return;
        }
        const uint64_t ts = (uint64_t)t * TP;
        const uint64_t te = ts + TP < s ? ts + TP : s;
        const uint64_t a0 = ts > b1 ? ts : b1;
        const uint32_t le = (t == tb ? w.x - eq_part : w.x) + w.y;
        const uint64_t aend = te < b2 ? te : b2;
        const uint32_t szA = aend > a0 ? (uint32_t)(aend - a0) : 0;
        const bool hasB = te > (ts > b2 ? ts : b2);
        const uint32_t leA = !hasB ? le : (szA == 0 ? 0 : eq_part2);
        *l = szA - leA;
        *r = le - leA;
    };
    const uint32_t X = scan_misplaced<NTH>(nt, ld, mis, preL, preR, stage, tmp);
    const uint32_t rc = rank_chunk(X, s, span);
    const uint32_t nch = (uint32_t)chunk_count(X, s, span);
    uint32_t *spL = spL_all + g.chunk_off, *spR = spR_all + g.chunk_off;
    mark_chunk_tiles<NTH>(nt, TP, rc, nch, preL, preR, spL, spR);
    if (threadIdx.x == 0) {
        meta[M_RCB] = rc;
        meta[M_XB] = X;
        spL[0] = (uint32_t)b1;
        spL[nch] = (uint32_t)b2;
        spR[0] = (uint32_t)b2;
        spR[nch] = (uint32_t)s;
    }
}
// One item per segment of the table.
template <class O, int NTH, bool LOOP>
__global__ __launch_bounds__(NTH) void k_part_scan_b(TaskRef<PartSeg> tasks, uint32_t first,
                                                     uint32_t TP, uint32_t span,
                                                     const uint32_t *cnt_eq_all,
                                                     const uint32_t *eqmv_all,
                                                     uint32_t *preL_all, uint32_t *preR_all,
                                                     uint32_t *spL_all, uint32_t *spR_all,
                                                     uint64_t *meta_all) {
    __shared__ ScanBLds<NTH> lds_mem;
    ScanBLds<NTH> *lds = &lds_mem;
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) part_scan_b_item<O, NTH>(tasks, item, TP, span, cnt_eq_all, eqmv_all, preL_all,
                                     preR_all, spL_all, spR_all, meta_all, *lds);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            part_scan_b_item<O, NTH>(tasks, item, TP, span, cnt_eq_all, eqmv_all, preL_all,
                                     preR_all, spL_all, spR_all, meta_all, *lds);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}

// Left region and right region of a pass, as offsets from the range start,
// and the class test: an element belongs left if ord(k) < p (pass A) or
// ord(k) <= p (pass B).
struct PassGeom {
    uint64_t l0, l1, r0, r1;
};
template <int PASS>
__device__ __forceinline__ PassGeom pass_geom(const uint64_t *meta, uint64_t s) {
    const uint64_t b1 = meta[M_CLT];
    PassGeom g;
    if (PASS == 0) {
        g.l0 = 0;
        g.l1 = b1;
        g.r0 = b1;
        g.r1 = s;
    } else {
        const uint64_t b2 = b1 + meta[M_CEQ];
        g.l0 = b1;
        g.l1 = b2;
        g.r0 = b2;
        g.r1 = s;
    }
    return g;
}
template <class O, int PASS, class K>
__device__ __forceinline__ bool belongs_left(K k, K p) {
    return PASS == 0 ? O::lt(k, p) : !O::lt(p, k);
}

// ---- split: position of the first misplaced element of every chunk ----------
// One wave per (chunk boundary j >= 1, side).  The scan recorded the tile
// holding the boundary and its rank k inside the tile; the wave finds the k-th
// misplaced element of the tile's part of the region and replaces the record
// with its position.  The host gives each segment an upper bound of
// 2 (chunks - 1) waves; surplus waves return.  In pass A, with the count's
// per-64 counts (`gcnt`) and a tile wholly inside the region, a wave scan
// over those counts picks the 64 positions that hold the element and one
// ballot over them finishes; otherwise the wave walks the tile.
template <class O, int PASS>
__device__ __forceinline__ void part_split_item(TaskRef<PartSeg> tasks, uint32_t gw,
                                                uint32_t TP, uint32_t *spL_all,
                                                uint32_t *spR_all, const uint8_t *gcnt,
                                                const uint64_t *meta_all) {
    uint32_t w, a;
    const PartSeg g = task_of_wave(tasks, gw, &w, &a);
    const uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
    const uint32_t X = (uint32_t)meta[PASS == 0 ? M_XA : M_XB];
    const uint32_t rc = (uint32_t)meta[PASS == 0 ? M_RCA : M_RCB];
    if (X == 0) return;
    const uint32_t nch = (X + rc - 1) / rc;
    const uint64_t j = 1 + w / 2;
    const int side = (int)(w & 1);
    if (j >= nch) return;
    using K = typename O::K;
    const K *keys = (const K *)g.keys + g.lo;
    const K p = (K)meta[M_PIVOT];
    const uint64_t s = g.s;
    const PassGeom geo = pass_geom<PASS>(meta, s);
    uint32_t *sp = (side ? spR_all : spL_all) + g.chunk_off;
    const uint32_t rec = sp[j];
    const uint32_t t = rec / TP;
    uint32_t k = rec - t * TP;
    const uint64_t ts = (uint64_t)t * TP;
    const uint64_t te = ts + TP < s ? ts + TP : s;
    const uint64_t reg0 = side ? geo.r0 : geo.l0, reg1 = side ? geo.r1 : geo.l1;
    uint64_t x0 = ts > reg0 ? ts : reg0;
    uint64_t x1 = te < reg1 ? te : reg1;
    const int lane = lane_id();
    if (PASS == 0 && gcnt != nullptr && x0 == ts && x1 == te) {
        // misplaced elements per 64 positions: #(< p) on the right side,
        // the rest on the left
        const uint8_t *gc = gcnt + ((uint64_t)g.tile_off + t) * (TP / kWave);
        const uint32_t ng = (uint32_t)((te - ts + kWave - 1) / kWave);
        for (uint32_t g0 = 0; g0 < ng; g0 += kWave) {
            const uint32_t gi = g0 + (uint32_t)lane;
            uint32_t c = 0;
            if (gi < ng) {
                const uint32_t less = gc[gi];
                const uint64_t len = te - ts - (uint64_t)gi * kWave;
                c = side ? less : (uint32_t)(len < kWave ? len : kWave) - less;
            }
            const uint32_t inc = wave_inclusive_scan(c);
            const uint32_t tot = (uint32_t)__shfl((int)inc, kWave - 1);
            if (k < tot) {
                const int hit = __ffsll((unsigned long long)__ballot(inc > k)) - 1;
                k -= (uint32_t)__shfl((int)(inc - c), hit);
                const uint64_t a0 = ts + (uint64_t)(g0 + (uint32_t)hit) * kWave;
                const uint64_t pos = a0 + (uint64_t)lane;
                const bool in = pos < te;
                const bool bl = belongs_left<O, PASS>(O::ord(ldg(keys + (in ? pos : te - 1))), p);
                const uint64_t m = __ballot(in && (side ? bl : !bl));
                if (((m >> lane) & 1ull) && (uint32_t)__popcll(m & lanemask_lt()) == k)
                    sp[j] = (uint32_t)pos;
                return;
            }
            k -= tot;
        }
        return;  // not reached: the tile holds more than k misplaced elements
    }
    // the wave walks the part 1024 positions a step, lane-interleaved
    // (coalesced loads, all in flight), and counts misplaced elements with
    // ballots
    constexpr int kQ = 16;
    for (uint64_t base = x0; base < x1; base += kWave * kQ) {
        K kv[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const uint64_t pos = base + (uint64_t)q * kWave + lane;
            kv[q] = ldg(keys + (pos < x1 ? pos : x1 - 1));
        }
        uint64_t m[kQ];
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const uint64_t pos = base + (uint64_t)q * kWave + lane;
            const bool bl = belongs_left<O, PASS>(O::ord(kv[q]), p);
            m[q] = __ballot(pos < x1 && (side ? bl : !bl));
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
            const uint32_t c = (uint32_t)__popcll(m[q]);
            if (k < c) {  // the k-th set bit of m[q]
                if (((m[q] >> lane) & 1ull) && (uint32_t)__popcll(m[q] & lanemask_lt()) == k)
                    sp[j] = (uint32_t)(base + (uint64_t)q * kWave + lane);
                return;
            }
            k -= c;
        }
    }
}
template <class O, int PASS, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_part_split(TaskRef<PartSeg> tasks, uint32_t first,
                                                       uint32_t TP, uint32_t total,
                                                       uint32_t *spL_all, uint32_t *spR_all,
                                                       const uint8_t *gcnt,
                                                       const uint64_t *meta_all) {
    // items: waves (no barriers)
    const uint32_t W = work_total(tasks, total);
    const uint32_t gw0 = first + blockIdx.x * kWaves + wave_id();
    if constexpr (!LOOP) {
        if (gw0 < W) part_split_item<O, PASS>(tasks, gw0, TP, spL_all, spR_all, gcnt, meta_all);
    } else {
        for (uint32_t gw = gw0; gw < W; gw += gridDim.x * kWaves)
            part_split_item<O, PASS>(tasks, gw, TP, spL_all, spR_all, gcnt, meta_all);
    }
}


// ---- swap ------------------------------------------------------------------------
// Scan state of one side of a chunk: its position range [pos, end) (offsets
// from the range start), the prefix counts of its tiles and the number of
// misplaced elements found so far.
struct SideScan {
    uint64_t pos, end;
    const uint32_t *pre;
    uint32_t found;
};

// Advance `sc.pos` past tiles whose prefix counts show no misplaced element
// (binary search for the next tile whose count grows).
__device__ __forceinline__ void skip_empty_tiles(SideScan &sc, uint32_t TP, uint32_t nt) {
    while (sc.pos < sc.end) {
        const uint64_t t = sc.pos / TP;
        const uint32_t pt = sc.pre[t];
        if (sc.pre[t + 1] != pt) return;
        uint64_t x = t + 1, y = nt;  // first i in (t, nt] with pre[i] > pt
        while (x < y) {
            const uint64_t mid = (x + y) >> 1;
            if (sc.pre[mid] > pt) y = mid;
            else x = mid + 1;
        }
        const uint64_t next = (x - 1) * TP;  // tile x - 1 holds the next element
        sc.pos = next > sc.pos ? next : (t + 1) * TP;
    }
}

// Load one subtile of kPartSub positions starting at sc.pos (wave-striped:
// wave w covers 16 x 64 consecutive positions, lane-interleaved; clamped
// loads, all in flight) and ballot its misplaced elements; the keys stay in
// kv for the exchange.
template <class O, int PASS>
__device__ __forceinline__ uint32_t ballot_subtile(const typename O::K *keys, typename O::K p,
                                                   bool right, const SideScan &sc,
                                                   uint64_t m[kPartItems],
                                                   typename O::K kv[kPartItems]) {
    const int lane = lane_id(), wave = wave_id();
    const uint64_t base = sc.pos + (uint64_t)wave * (kPartItems * kWave) + lane;
#pragma unroll
    for (int q = 0; q < kPartItems; ++q) {
        const uint64_t pos = base + (uint64_t)q * kWave;
        kv[q] = ldg(keys + (pos < sc.end ? pos : sc.end - 1));
    }
    uint32_t wcount = 0;
#pragma unroll
    for (int q = 0; q < kPartItems; ++q) {
        const uint64_t pos = base + (uint64_t)q * kWave;
        const bool bl = belongs_left<O, PASS>(O::ord(kv[q]), p);
        m[q] = __ballot(pos < sc.end && (right ? bl : !bl));
        wcount += (uint32_t)__popcll(m[q]);
    }
    return wcount;
}

// Record the positions of a subtile's misplaced elements in `slots` and
// their keys in `vslots`, in position order, after the waves' counts are
// known (wtot: one per wave).
template <class K>
__device__ __forceinline__ void record_subtile(SideScan &sc, const uint64_t m[kPartItems],
                                               const K kv[kPartItems],
                                               const uint32_t *wtot, uint32_t *slots,
                                               K *vslots, uint32_t cap) {
    const int lane = lane_id(), wave = wave_id();
    uint32_t woff = sc.found, total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) woff += wtot[w];
        total += wtot[w];
    }
    const uint64_t base = sc.pos + (uint64_t)wave * (kPartItems * kWave) + lane;
#pragma unroll
    for (int q = 0; q < kPartItems; ++q) {
        if ((m[q] >> lane) & 1ull) {
            const uint32_t slot = woff + (uint32_t)__popcll(m[q] & lanemask_lt());
            if (slot < cap) {  // always true with consistent counts
                slots[slot] = (uint32_t)(base + (uint64_t)q * kWave);
                vslots[slot] = kv[q];
            }
        }
        woff += (uint32_t)__popcll(m[q]);
    }
    sc.found += total;
    sc.pos += kPartSub;
}

// One workgroup per chunk: find the positions of the chunk's misplaced
// elements on both sides (the two ranges are scanned in the same steps, so
// their loads overlap), then exchange the k-th of the left with the k-th of
// the right.  Positions and keys are kept in LDS, so the exchange only
// stores (reading the keys again would fetch nearly every line of the range
// a second time: misplaced elements are dense when the pivot is central);
// payloads of key/payload sorts are gathered at the exchange.
struct SwapLds {
    uint32_t pL[kRankChunk], pR[kRankChunk];
    uint32_t wtot[2][kWaves];
};
template <class O, bool PAIRS, int PASS>
__device__ __forceinline__ void part_swap_item(TaskRef<PartSeg> tasks, uint32_t item,
                                               uint32_t TP, const uint32_t *preL_all,
                                               const uint32_t *preR_all,
                                               const uint32_t *spL_all,
                                               const uint32_t *spR_all, uint32_t *eqmv_all,
                                               const uint64_t *meta_all, SwapLds &lds,
                                               typename O::K *vL, typename O::K *vR) {
    using K = typename O::K;
    uint32_t *pL = lds.pL, *pR = lds.pR;
    uint32_t(*wtot)[kWaves] = lds.wtot;
    uint32_t j, a;
    const PartSeg g = task_of(tasks, item, &j, &a);
    const uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
    const uint32_t X = (uint32_t)meta[PASS == 0 ? M_XA : M_XB];
    const uint32_t rc = (uint32_t)meta[PASS == 0 ? M_RCA : M_RCB];
    if (X == 0) return;
    const uint32_t nch = (X + rc - 1) / rc;
    if (j >= nch) return;
    K *keys = (K *)g.keys + g.lo;
    uint32_t *vals = PAIRS ? g.vals + g.lo : nullptr;
    const K p = (K)meta[M_PIVOT];
    const uint32_t r0 = j * rc;
    uint32_t cnt = X - r0 < rc ? X - r0 : rc;
    const uint32_t *spL = spL_all + g.chunk_off, *spR = spR_all + g.chunk_off;
    // position ranges of this chunk, clamped to the pass's regions
    const PassGeom geo = pass_geom<PASS>(meta, g.s);
    SideScan L{spL[j] > geo.l0 ? spL[j] : geo.l0, spL[j + 1] < geo.l1 ? spL[j + 1] : geo.l1,
               preL_all + g.tile_off + g.slot, 0};
    SideScan R{spR[j] > geo.r0 ? spR[j] : geo.r0, spR[j + 1] < geo.r1 ? spR[j + 1] : geo.r1,
               preR_all + g.tile_off + g.slot, 0};
    // look for empty tiles only where the misplaced elements are sparse
    const bool sparse_l = L.end > L.pos && L.end - L.pos > 8ull * kPartSub + 8ull * cnt;
    const bool sparse_r = R.end > R.pos && R.end - R.pos > 8ull * kPartSub + 8ull * cnt;
    for (;;) {
        if (sparse_l) skip_empty_tiles(L, TP, g.nt);
        if (sparse_r) skip_empty_tiles(R, TP, g.nt);
        const bool more_l = L.pos < L.end, more_r = R.pos < R.end;
        if (!more_l && !more_r) break;
        // both sides' loads in flight together, one pair of barriers
        uint64_t mL[kPartItems], mR[kPartItems];
        K kL[kPartItems], kR[kPartItems];
        uint32_t cl = 0, cr = 0;
        if (more_l) cl = ballot_subtile<O, PASS>(keys, p, false, L, mL, kL);
        if (more_r) cr = ballot_subtile<O, PASS>(keys, p, true, R, mR, kR);
        if (lane_id() == 0) {
            wtot[0][wave_id()] = cl;
            wtot[1][wave_id()] = cr;
        }
        __syncthreads();
        if (more_l) record_subtile(L, mL, kL, wtot[0], pL, vL, kRankChunk);
        if (more_r) record_subtile(R, mR, kR, wtot[1], pR, vR, kRankChunk);
        __syncthreads();  // wtot is rewritten by the next step
    }
    __syncthreads();
    // equal by construction; the minimum keeps every access inside the filled slots
    cnt = min(cnt, min(L.found, R.found));
    if (cnt == 0) return;
    uint32_t *eqmv = eqmv_all + g.tile_off;
    // every thread exchanges up to kXItems pairs (clamped slots read a
    // valid pair and store nothing)
    constexpr int kXItems = (kRankChunk + kBlock - 1) / kBlock;
    uint32_t il[kXItems], ir[kXItems];
    K x[kXItems], y[kXItems];
#pragma unroll
    for (int q = 0; q < kXItems; ++q) {
        const uint32_t k = (uint32_t)q * kBlock + threadIdx.x;
        const uint32_t kk = k < cnt ? k : cnt - 1;
        il[q] = pL[kk];
        ir[q] = pR[kk];
        x[q] = vL[kk];
        y[q] = vR[kk];
    }
#pragma unroll
    for (int q = 0; q < kXItems; ++q) {
        const uint32_t k = (uint32_t)q * kBlock + threadIdx.x;
        if (k < cnt) {
            stg(keys + il[q], y[q]);
            stg(keys + ir[q], x[q]);
            if (PASS == 0 && O::ord(x[q]) == p) atomicAdd(&eqmv[ir[q] / TP], 1u);
        }
    }
    if constexpr (PAIRS) {
        uint32_t xv[kXItems], yv[kXItems];
#pragma unroll
        for (int q = 0; q < kXItems; ++q) {
            xv[q] = ldg(vals + il[q]);
            yv[q] = ldg(vals + ir[q]);
        }
#pragma unroll
        for (int q = 0; q < kXItems; ++q) {
            const uint32_t k = (uint32_t)q * kBlock + threadIdx.x;
            if (k < cnt) {
                stg(vals + il[q], yv[q]);
                stg(vals + ir[q], xv[q]);
            }
        }
    }
}
template <class O, bool PAIRS, int PASS, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_part_swap(TaskRef<PartSeg> tasks, uint32_t first,
                                                      uint32_t TP, const uint32_t *preL_all,
                                                      const uint32_t *preR_all,
                                                      const uint32_t *spL_all,
                                                      const uint32_t *spR_all,
                                                      uint32_t *eqmv_all,
                                                      const uint64_t *meta_all) {
    using K = typename O::K;
    __shared__ SwapLds lds_mem;
    __shared__ K vL_mem[kRankChunk], vR_mem[kRankChunk];
    SwapLds *lds = &lds_mem;
    K *vL = vL_mem, *vR = vR_mem;
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) part_swap_item<O, PAIRS, PASS>(tasks, item, TP, preL_all, preR_all, spL_all,
                                           spR_all, eqmv_all, meta_all, *lds, vL, vR);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            part_swap_item<O, PAIRS, PASS>(tasks, item, TP, preL_all, preR_all, spL_all,
                                           spR_all, eqmv_all, meta_all, *lds, vL, vR);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}


// ---- host side ---------------------------------------------------------------------
template <class O, bool PAIRS, bool LOOP>
static hipError_t partition_phase(const PartitionLaunch &L, hipStream_t st) {
    const Workspace &ws = *L.ws;
    // L.grid workgroups from item L.first on: exactly the work items of a
    // host-sized launch; for a device-sized one the estimate (first = 0) or
    // the overflow (LOOP)
    if (L.grid == 0) return hipSuccess;
    const uint32_t f = L.first;
    switch (L.phase) {
    case 0: {  // count
        ProfScope prof(st, K_PART_COUNT, (double)sizeof(typename O::K) * L.keys_total);
        hipLaunchKernelGGL((k_part_count<O, LOOP>), dim3(L.grid), dim3(kBlock), 0, st, L.tasks, f,
                           L.TP, ws.cnt_lt, ws.cnt_eq, L.groups ? ws.gcnt : nullptr,
                           (const uint64_t *)ws.meta);
        break;
    }
    case 6: {  // scan A (tasks.pre counts each segment's scan workgroups)
        ProfScope prof(st, K_PART_SCAN, 0.0);
        if (L.scan_threads == kScanThreads)
            hipLaunchKernelGGL((k_part_scan_a<O, kScanThreads, LOOP>), dim3(L.grid),
                               dim3(kScanThreads), 0, st, L.tasks, f, L.TP, L.chunk_span,
                               ws.cnt_lt, ws.cnt_eq, ws.preL, ws.preR, ws.eqmv, ws.spL, ws.spR,
                               ws.meta, ws.res);
        else
            hipLaunchKernelGGL((k_part_scan_a<O, kBlock, LOOP>), dim3(L.grid), dim3(kBlock), 0, st,
                               L.tasks, f, L.TP, L.chunk_span, ws.cnt_lt, ws.cnt_eq, ws.preL,
                               ws.preR, ws.eqmv, ws.spL, ws.spR, ws.meta, ws.res);
        break;
    }
    case 1:    // split of pass A
    case 3: {  // split of pass B (items: waves; L.work: waves of a host-sized launch)
        ProfScope prof(st, K_PART_SPLIT, 0.0);
        if (L.phase == 1)
            hipLaunchKernelGGL((k_part_split<O, 0, LOOP>), dim3(L.grid), dim3(kBlock), 0, st,
                               L.tasks, f, L.TP, L.work, ws.spL, ws.spR,
                               L.groups ? ws.gcnt : nullptr, (const uint64_t *)ws.meta);
        else
            hipLaunchKernelGGL((k_part_split<O, 1, LOOP>), dim3(L.grid), dim3(kBlock), 0, st,
                               L.tasks, f, L.TP, L.work, ws.spL, ws.spR,
                               (const uint8_t *)nullptr, (const uint64_t *)ws.meta);
        break;
    }
    case 2:    // swap of pass A
    case 5: {  // swap of pass B (its pair count is known only on the device)
        ProfScope prof(st, K_PART_SWAP, L.phase == 2 ? L.bytes : 0.0);
        if (L.phase == 2)
            hipLaunchKernelGGL((k_part_swap<O, PAIRS, 0, LOOP>), dim3(L.grid), dim3(kBlock), 0, st,
                               L.tasks, f, L.TP, ws.preL, ws.preR, ws.spL, ws.spR, ws.eqmv,
                               (const uint64_t *)ws.meta);
        else
            hipLaunchKernelGGL((k_part_swap<O, PAIRS, 1, LOOP>), dim3(L.grid), dim3(kBlock), 0, st,
                               L.tasks, f, L.TP, ws.preL, ws.preR, ws.spL, ws.spR, ws.eqmv,
                               (const uint64_t *)ws.meta);
        break;
    }
    case 4: {  // scan B, one item per segment
        ProfScope prof(st, K_PART_SCAN, 0.0);
        if (L.scan_threads == kScanThreads)
            hipLaunchKernelGGL((k_part_scan_b<O, kScanThreads, LOOP>), dim3(L.grid),
                               dim3(kScanThreads), 0, st, L.tasks, f, L.TP, L.chunk_span,
                               ws.cnt_eq, ws.eqmv, ws.preL, ws.preR, ws.spL, ws.spR, ws.meta);
        else
            hipLaunchKernelGGL((k_part_scan_b<O, kBlock, LOOP>), dim3(L.grid), dim3(kBlock), 0, st,
                               L.tasks, f, L.TP, L.chunk_span, ws.cnt_eq, ws.eqmv, ws.preL,
                               ws.preR, ws.spL, ws.spR, ws.meta);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
template <class O, bool PAIRS>
static hipError_t partition_t(const PartitionLaunch &L, hipStream_t st) {
    return L.loop ? partition_phase<O, PAIRS, true>(L, st) : partition_phase<O, PAIRS, false>(L, st);
}

hipError_t launch_partition_phase(int dt, bool pairs, const PartitionLaunch &L, hipStream_t st) {
    switch (dt) {
    case 0:
        return pairs ? partition_t<OrdU32, true>(L, st) : partition_t<OrdU32, false>(L, st);
    case 1:
        return pairs ? partition_t<OrdF32, true>(L, st) : partition_t<OrdF32, false>(L, st);
    case 2:
        return pairs ? partition_t<OrdU64, true>(L, st) : partition_t<OrdU64, false>(L, st);
    case 3:
        return pairs ? partition_t<OrdF64, true>(L, st) : partition_t<OrdF64, false>(L, st);
    case 4:
        return pairs ? hipErrorInvalidValue : partition_t<OrdLogU32, false>(L, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace qms
