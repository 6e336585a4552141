// qms_merge.hip -- one level of the swap-merge on gfx950.
//
// Fig. 2's merge takes two sorted runs and writes their merge into a target
// area, moving the elements found in the target into the cells the runs
// vacate (Sec. "QuickXsort and QuickMergesort": an element Mergesort would
// move to extra space is swapped with the element occupying that cell).
//
// Here a level merges consecutive pairs of runs of width W of a source
// region S into the destination region D of the same length (S and D are the
// data side and the buffer side of the current partition round, in either
// order).  The output of each pair is cut into tiles of kMergeTile elements;
// the merge-path split (the diagonal search of Odeh et al.'s Merge Path) gives
// every tile its own slice of each run, disjoint from every other tile's
// slices.  A workgroup therefore reads its two run slices and its output
// window of D, writes the merged keys into the window and the displaced
// window contents into the run-slice cells it just read.  No workgroup
// touches another's cells.  The splits are found by a separate kernel before
// the level starts: a search inside the merge kernel would probe run cells
// that neighbouring workgroups are already overwriting with buffer elements.
// The split array (one word per tile) is part of the fixed-size workspace.
// Ties go to the left run.
#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

namespace qms {

// Geometry of merge tile `tile` of a level: run pair base, lengths, diagonals.
struct MergeTileGeom {
    uint64_t pb, lenA, lenB, d0, d1;
};
__device__ __forceinline__ MergeTileGeom merge_geom(uint64_t m, uint64_t W, uint64_t tile) {
    MergeTileGeom g;
    const uint64_t start = tile * kMergeTile;
    g.pb = (start / (2 * W)) * (2 * W);
    g.d0 = start - g.pb;
    const uint64_t rest = m - g.pb;
    g.lenA = rest < W ? rest : W;
    g.lenB = rest > W ? (rest - W < W ? rest - W : W) : 0;
    const uint64_t tot = g.lenA + g.lenB;
    g.d1 = g.d0 + kMergeTile < tot ? g.d0 + kMergeTile : tot;
    return g;
}

// Regions of a merge level: the base case leaves the runs in R0 (the buffer
// when the level count is odd, the data region otherwise); level l reads
// R(l mod 2) and writes the other region, so the last level ends in D.
__device__ __forceinline__ void level_regions(const SortSeg &g, uint32_t level, uint32_t *src,
                                              uint32_t *dst) {
    const bool odd = (g.L & 1u) != 0;
    const uint32_t r0 = odd ? g.Bf : g.D, r1 = odd ? g.D : g.Bf;
    *src = (level & 1u) ? r1 : r0;
    *dst = (level & 1u) ? r0 : r1;
}

// First index in [lo, hi) where the prefix-true predicate pred fails (hi if
// it holds everywhere), searched by kSplitLanes lanes together: each step the
// lanes probe kSplitLanes evenly spaced candidates and a ballot narrows the
// range kSplitLanes-fold.  Fewer dependent steps than a binary search for a
// few more probes.  Every lane of the wave calls it; inactive groups pass an
// empty range.
template <class F>
__device__ __forceinline__ uint64_t group_first_false(uint64_t lo, uint64_t hi, F pred) {
    constexpr uint32_t G = kSplitLanes;
    const uint32_t sub = lane_id() % G;
    const uint32_t gshift = (lane_id() / G) * G;
    // every lane of the wave loops while any group still searches
    while (__ballot(hi > lo) != 0) {
        const uint64_t step = hi > lo ? (hi - lo + G - 1) / G : 1;
        const uint64_t i = lo + (uint64_t)sub * step;
        const bool t = i < hi && pred(i);
        const uint64_t bits = (__ballot(t) >> gshift) & ((1ull << G) - 1);
        const int c = __popcll(bits);
        if (hi > lo) {
            const uint64_t nlo = c > 0 ? lo + (uint64_t)(c - 1) * step + 1 : lo;
            const uint64_t cand = lo + (uint64_t)c * step;
            hi = cand < hi ? cand : hi;
            lo = nlo;
        }
    }
    return lo;
}

// kSplitLanes lanes per merge tile: the merge-path split at the tile's first
// output d, i.e. the number c of elements of run A among the first d outputs
// (c = the first i with A[i] > B[d - 1 - i], within the diagonal's range
// [lo, hi]).  The search runs in two stages:
//   coarse  on the samples of the runs (every kMergeTile-th element, written
//           by the previous level or the base case; a small array that stays
//           in cache): with S = kMergeTile and d a multiple of S, the test
//           Q(u): uS <= hi and (d - uS >= |B| or A[(u-1)S] <= B[d - uS])
//           only reads samples, holds whenever c >= uS, and is prefix-true;
//           for the last u1 with Q(u1), (u1 - 1) S < c < (u1 + 1) S;
//   fine    on the runs, inside that window of fewer than 2S candidates.
// The 4-lane searches beat both a one-lane binary search (latency) and a
// wave-wide one (cache lines touched) once there are thousands of splits.
template <class O>
__global__ __launch_bounds__(kBlock) void k_merge_split(TaskRef<SortSeg> tasks, uint32_t level,
                                                        uint32_t total, uint32_t *splits,
                                                        const uint32_t *samples) {
    constexpr uint64_t S = kMergeTile;
    const uint32_t gid = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t w = gid / kSplitLanes;
    const bool active = w < total;
    uint32_t tile = 0, a = 0;
    const SortSeg g = task_of(tasks, active ? w : total - 1, &tile, &a);
    uint32_t src, dst;
    level_regions(g, level, &src, &dst);
    const uint64_t W = (uint64_t)g.w0 << level;
    const MergeTileGeom geo = merge_geom(g.m, W, tile);
    const uint32_t *A = g.keys + src + geo.pb;
    const uint32_t *B = A + W;
    const uint32_t *As = samples + g.split_off + geo.pb / S;
    const uint32_t *Bs = As + W / S;
    const uint64_t d = geo.d0, nA = geo.lenA, nB = geo.lenB;
    uint64_t lo = d > nB ? d - nB : 0;
    uint64_t hi = d < nA ? d : nA;
    if (!active) lo = hi = 0;
    // coarse: first u in [1, hi / S] without Q(u)
    const uint64_t f = group_first_false(1, active ? hi / S + 1 : 1, [&](uint64_t u) {
        return d - u * S >= nB || ldg(As + u - 1) <= ldg(Bs + (d - u * S) / S);
    });
    const uint64_t u1 = f - 1;
    const uint64_t wl = u1 >= 1 ? max(lo, (u1 - 1) * S + 1) : lo;
    const uint64_t wh = min(hi, (u1 + 1) * S - 1);
    // fine: the first i in [wl, wh) with A[i] > B[d - 1 - i], else wh
    const uint64_t c = group_first_false(wl, wh, [&](uint64_t i) {
        return O::ord(ldg(A + i)) <= O::ord(ldg(B + d - 1 - i));
    });
    if (active && gid % kSplitLanes == 0) splits[g.split_off + tile] = (uint32_t)c;
}

template <class O, bool PAIRS>
__device__ __forceinline__ void merge_block(uint32_t *S, uint32_t *SV, uint32_t *D,
                                            uint32_t *DV, uint64_t m, uint64_t W,
                                            uint64_t tile, const uint32_t *splits,
                                            uint32_t *samples_out) {
    __shared__ uint32_t sk[kMergeTile];
    __shared__ uint32_t sv[PAIRS ? kMergeTile : 1];
    const uint32_t tid = threadIdx.x;

    const MergeTileGeom g = merge_geom(m, W, tile);
    const uint64_t pb = g.pb, d0 = g.d0, d1 = g.d1;
    const uint32_t cnt = (uint32_t)(d1 - d0);
    // splits as found by k_merge_split, clamped to the ranges a merge path
    // can take (a no-op for consistent splits; keeps every access in the runs)
    uint64_t i0 = splits[tile];
    uint64_t i1 = d1 < g.lenA + g.lenB ? (uint64_t)splits[tile + 1] : g.lenA;
    i0 = min(max(i0, d0 > g.lenB ? d0 - g.lenB : 0), min(d0, g.lenA));
    i1 = min(max(i1, max(i0, d1 > g.lenB ? d1 - g.lenB : 0)), min(min(d1, g.lenA), i0 + cnt));

    // the destination window's current contents (buffer elements)
    // clamped, unconditional loads so that all of them are in flight together
    uint32_t oldk[kMergePerThread];
    uint32_t oldv[PAIRS ? kMergePerThread : 1];
#pragma unroll
    for (int q = 0; q < kMergePerThread; ++q) {
        const uint32_t e = min((uint32_t)(q * kBlock + tid), cnt - 1);
        oldk[q] = ldg(D + pb + d0 + e);
        if constexpr (PAIRS) oldv[q] = ldg(DV + pb + d0 + e);
    }
    const uint64_t j0 = d0 - i0, j1 = d1 - i1;
    const uint32_t na = (uint32_t)(i1 - i0);
    const uint32_t nb = (uint32_t)(j1 - j0);
    uint32_t nk[kMergePerThread];
    uint32_t nv[PAIRS ? kMergePerThread : 1];
#pragma unroll
    for (int q = 0; q < kMergePerThread; ++q) {
        const uint32_t e = min((uint32_t)(q * kBlock + tid), cnt - 1);
        const uint64_t pos = e < na ? pb + i0 + e : pb + W + j0 + (e - na);
        nk[q] = ldg(S + pos);
        if constexpr (PAIRS) nv[q] = ldg(SV + pos);
    }
#pragma unroll
    for (int q = 0; q < kMergePerThread; ++q) {
        const uint32_t e = q * kBlock + tid;
        if (e < cnt) {
            sk[e] = O::ord(nk[q]);
            if constexpr (PAIRS) sv[e] = nv[q];
        }
    }
    __syncthreads();

    // each thread merges kMergePerThread consecutive outputs of the tile
    uint32_t ok[kMergePerThread];
    uint32_t ov[PAIRS ? kMergePerThread : 1];
    const uint32_t diag = tid * kMergePerThread;
    if (diag < cnt) {
        uint32_t lo = diag > nb ? diag - nb : 0;
        uint32_t hi = diag < na ? diag : na;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (sk[mid] <= sk[na + diag - 1 - mid]) lo = mid + 1;
            else hi = mid;
        }
        uint32_t ia = lo, ib = diag - lo;
        uint32_t ka = ia < na ? sk[ia] : 0u;
        uint32_t kb = ib < nb ? sk[na + ib] : 0u;
#pragma unroll
        for (int q = 0; q < kMergePerThread; ++q) {
            if (diag + q < cnt) {
                const bool takeA = ib >= nb || (ia < na && ka <= kb);
                if (takeA) {
                    ok[q] = ka;
                    if constexpr (PAIRS) ov[q] = sv[ia];
                    ++ia;
                    ka = ia < na ? sk[ia] : 0u;
                } else {
                    ok[q] = kb;
                    if constexpr (PAIRS) ov[q] = sv[na + ib];
                    ++ib;
                    kb = ib < nb ? sk[na + ib] : 0u;
                }
            }
        }
    }
    __syncthreads();
    if (diag < cnt) {
#pragma unroll
        for (int q = 0; q < kMergePerThread; ++q) {
            if (diag + q < cnt) {
                sk[diag + q] = ok[q];
                if constexpr (PAIRS) sv[diag + q] = ov[q];
            }
        }
    }
    __syncthreads();
    // the tile's first output is the sample the next level's split search uses
    if (tid == 0) stg(samples_out + tile, sk[0]);
#pragma unroll
    for (int q = 0; q < kMergePerThread; ++q) {
        const uint32_t e = q * kBlock + tid;
        if (e < cnt) {
            stg(D + pb + d0 + e, O::unord(sk[e]));
            if constexpr (PAIRS) stg(DV + pb + d0 + e, sv[e]);
            const uint64_t pos = e < na ? pb + i0 + e : pb + W + j0 + (e - na);
            stg(S + pos, oldk[q]);
            if constexpr (PAIRS) stg(SV + pos, oldv[q]);
        }
    }
}

template <class O, bool PAIRS>
__global__ __launch_bounds__(kBlock) void k_merge(TaskRef<SortSeg> tasks, uint32_t level,
                                                  const uint32_t *splits,
                                                  uint32_t *samples_out) {
    uint32_t tile, a;
    const SortSeg g = task_of(tasks, blockIdx.x, &tile, &a);
    if (tile * (uint64_t)kMergeTile >= g.m) return;
    uint32_t src, dst;
    level_regions(g, level, &src, &dst);
    merge_block<O, PAIRS>(g.keys + src, PAIRS ? g.vals + src : nullptr, g.keys + dst,
                          PAIRS ? g.vals + dst : nullptr, g.m, (uint64_t)g.w0 << level,
                          tile, splits + g.split_off, samples_out + g.split_off);
}

template <class O, bool PAIRS>
static hipError_t merge_t(const TaskRef<SortSeg> &tasks, uint32_t level, uint32_t tiles,
                          double bytes, const Workspace &ws, hipStream_t st) {
    if (tiles == 0) return hipSuccess;
    // level l searches the samples written by level l - 1 (or the base case)
    // and writes the other array
    const uint32_t *smp_in = ws.samples[level & 1];
    uint32_t *smp_out = ws.samples[(level + 1) & 1];
    {
        ProfScope prof(st, K_MERGE_SPLIT, 0.0);
        const uint64_t threads = (uint64_t)tiles * kSplitLanes;
        hipLaunchKernelGGL((k_merge_split<O>), dim3((uint32_t)((threads + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, tasks, level, tiles, ws.splits, smp_in);
    }
    {
        // per element: read the run cell and the window cell, write both
        ProfScope prof(st, K_MERGE, bytes);
        hipLaunchKernelGGL((k_merge<O, PAIRS>), dim3(tiles), dim3(kBlock), 0, st, tasks, level,
                           (const uint32_t *)ws.splits, smp_out);
    }
    return hipGetLastError();
}

hipError_t launch_merge_level(int dt, bool pairs, const TaskRef<SortSeg> &tasks, uint32_t level,
                              uint32_t tiles, double bytes, const Workspace &ws, hipStream_t st) {
    if (dt == 1)
        return pairs ? merge_t<OrdF32, true>(tasks, level, tiles, bytes, ws, st)
                     : merge_t<OrdF32, false>(tasks, level, tiles, bytes, ws, st);
    return pairs ? merge_t<OrdU32, true>(tasks, level, tiles, bytes, ws, st)
                 : merge_t<OrdU32, false>(tasks, level, tiles, bytes, ws, st);
}

}  // namespace qms
