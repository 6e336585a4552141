// qms_merge.hip -- the swap-merge passes of the Mergesort on gfx950.
//
// Fig. 2's merge takes two sorted runs and writes their merge into a target
// area, moving the elements found in the target into the cells the runs
// vacate (Sec. "QuickXsort and QuickMergesort": an element Mergesort would
// move to extra space is swapped with the element occupying that cell).
//
// 2-way pass: consecutive pairs of runs of width W of a source region S are
// merged into the destination region D of the same length (S and D are the
// data side and the buffer side of the current partition round, in either
// order).  The output of each pair is cut into tiles of kMergeTile elements;
// the merge-path split (the diagonal search of Odeh et al.'s Merge Path) gives
// every tile its own slice of each run, disjoint from every other tile's
// slices.  A workgroup reads its two run slices and its output window of D,
// writes the merged keys into the window and the displaced window contents
// into the run-slice cells it just read.  No workgroup touches another's
// cells.  The splits are found by a separate kernel before the pass starts: a
// search inside the merge kernel would probe run cells that neighbouring
// workgroups are already overwriting with buffer elements.
//
// 4-way pass (the multi-way merging the paper's conclusion proposes): groups of four runs A, B, C, D are merged at once, so a pass
// moves every element once for two levels of the binary Mergesort.  Its
// tiles are bounded by exact boundaries that need no multi-way search: the
// pair splits of (A, B) and (C, D) at every kMergeTile-th element give the
// elements x = AB[k kMergeTile] and y = CD[j kMergeTile] with their places
// in their pair, and the place of x among C and D is #(C < x) + #(D < x)
// (ties go to A, then B, then C, then D), of y among A and B #(A <= y) +
// #(B <= y): two plain searches each.  A tile runs from one boundary to the
// next in merge order; it holds at most kMergeTile elements of each pair
// (kMergeTile + kMerge4Absorb when it absorbs a tiny tile, see below).
// The workgroup merges A with B and C with D in LDS, then the two results.
//
// Ties go to the earlier run.  The split arrays (one entry per tile) and the
// run samples the searches start from are part of the fixed-size workspace.
#include <type_traits>

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

// Regions of a merge pass: the base case leaves the runs in R0 (the buffer
// when the pass count is odd, the data region otherwise); pass p reads
// R(p mod 2) and writes the other region, so the last pass ends in D.
struct Regions {
    uint32_t *sk, *sv;  // source keys, payloads
    uint32_t *dk, *dv;  // destination keys, payloads
};
__device__ __forceinline__ Regions level_regions(const SortSeg &g, uint32_t level) {
    const bool odd = (merge_passes(g.L, g.two_way != 0) & 1u) != 0;
    const bool p1 = (pass_index(g.L, level, g.two_way != 0) & 1u) != 0;
    // the region holding the runs at this pass: R0 on even passes
    const bool from_buffer = odd != p1;
    Regions r;
    r.sk = from_buffer ? g.bkeys : g.keys;
    r.sv = from_buffer ? g.bvals : g.vals;
    r.dk = from_buffer ? g.keys : g.bkeys;
    r.dv = from_buffer ? g.vals : g.bvals;
    return r;
}

// The binary level a launch works on for task g: `level` itself, or with
// `step` (device-sized rounds, where one launch runs the k-th pass of every
// task whatever its level count) the level of the task's k-th pass (k =
// level): 2k for an even level count, 2k + 1 for an odd one (its first pass,
// a 2-way one at level 0, runs in a launch of its own), k for 2-way tasks.
__device__ __forceinline__ uint32_t task_level(const SortSeg &g, uint32_t level, uint32_t step) {
    if (!step) return level;
    return g.two_way ? level : 2 * level + (g.L & 1u);
}
// Run samples: pass p of a task reads the array of its parity and writes
// the other one (the base case writes array 0 for pass 0).
template <class K>
__device__ __forceinline__ const K *samples_in(const SortSeg &g, uint32_t level, K *s0, K *s1) {
    return (pass_index(g.L, level, g.two_way != 0) & 1u) ? s1 : s0;
}
template <class K>
__device__ __forceinline__ K *samples_out(const SortSeg &g, uint32_t level, K *s0, K *s1) {
    return (pass_index(g.L, level, g.two_way != 0) & 1u) ? s0 : s1;
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
//   coarse  on the samples of the runs (every kSampleStride-th element,
//           written by the previous level or the base case; a small array
//           that stays in cache): with S = kSampleStride and d a multiple of
//           S (d is a multiple of kMergeTile), the test
//           Q(u): uS <= hi and (d - uS >= |B| or A[(u-1)S] <= B[d - uS])
//           only reads samples, holds whenever c >= uS, and is prefix-true;
//           for the last u1 with Q(u1), (u1 - 1) S < c < (u1 + 1) S;
//   fine    on the runs, inside that window of fewer than 2S candidates.
// The 4-lane searches beat both a one-lane binary search (latency) and a
// wave-wide one (cache lines touched) once there are thousands of splits.
// Geometry of pair tile `tile` in a 4-way pass over runs of width W: the group
// base gb (a multiple of 4W), which pair (0: A,B; 1: C,D), the tile's index k
// within its pair, and the four run lengths.
struct Merge4Geom {
    uint64_t gb;
    uint32_t which, k;
    uint32_t n[4];
};
__device__ __forceinline__ Merge4Geom merge4_geom(uint64_t m, uint64_t W, uint64_t tile) {
    Merge4Geom g;
    const uint64_t start = tile * kMergeTile;
    g.gb = (start / (4 * W)) * (4 * W);
    g.which = (uint32_t)((start - g.gb) / (2 * W));
    g.k = (uint32_t)((start - g.gb - g.which * 2 * W) / kMergeTile);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t b = g.gb + r * W;
        g.n[r] = b >= m ? 0u : (uint32_t)(m - b < W ? m - b : W);
    }
    return g;
}

// Number of elements of the sorted run Y (nY elements, samples Ys of every
// kSampleStride-th one) that precede x: #(Y < x) if strict, else #(Y <= x).
// First on the samples (u of them precede x, so the count lies in
// [(u-1) S + 1, u S]), then inside that gap.  A group collective (every
// lane of the wave calls it; inactive groups pass nY = 0).
template <class O>
__device__ __forceinline__ uint64_t group_count_before(const typename O::K *Y,
                                                       const typename O::K *Ys, uint64_t nY,
                                                       typename O::K x, bool strict) {
    using K = typename O::K;
    constexpr uint64_t S = kSampleStride;
    auto before = [&](K v) { return strict ? O::lt(v, x) : !O::lt(x, v); };
    const uint64_t u =
        group_first_false(0, (nY + S - 1) / S, [&](uint64_t i) { return before(ldg(Ys + i)); });
    const uint64_t lo = u == 0 ? 0 : (u - 1) * S + 1;
    const uint64_t hi = u == 0 ? 0 : min(u * S, nY);
    return group_first_false(lo, hi, [&](uint64_t i) { return before(O::ord(ldg(Y + i))); });
}

// With BOUNDS (the first step of a 4-way pass over runs A, B, C, D) each tile
// has two groups; both find the split (the same result, found in parallel),
// take the element at it, x = AB[d] (or CD[d]), and each counts its
// predecessors in one run of the other pair: #(C < x) and #(D < x) for a
// boundary of (A, B) (ties go to A, B first), #(A <= x) and #(B <= x) for
// one of (C, D).  The tile's start vector (4 words) goes to bounds.
template <class O, bool PAIRS, bool BOUNDS>
__device__ __forceinline__ void merge_split_item(TaskRef<SortSeg> tasks, uint32_t gid,
                                                 uint32_t total, uint32_t level_arg,
                                                 uint32_t step, uint32_t *splits,
                                                 typename O::K *samples0,
                                                 typename O::K *samples1, uint32_t *bounds) {
    using K = typename O::K;
    constexpr uint64_t S = kSampleStride;
    constexpr uint32_t GPT = BOUNDS ? 2 : 1;  // lane groups per tile
    const uint32_t w = gid / (GPT * kSplitLanes);
    const uint32_t half = (gid / kSplitLanes) % GPT;
    const bool active = w < total;
    uint32_t tile = 0, a = 0;
    const SortSeg g = task_of_lanes(tasks, active ? w : total - 1, &tile, &a);
    const uint32_t level = task_level(g, level_arg, step);
    const K *samples = samples_in<K>(g, level, samples0, samples1);
    const Regions rg = level_regions(g, level);
    const uint64_t W = (uint64_t)g.w0 << level;
    const MergeTileGeom geo = merge_geom(g.m, W, tile);
    const K *A = (const K *)rg.sk + geo.pb;
    const K *B = A + W;
    // the task's samples start at kSamplesPerTile entries per split tile
    const K *smp = samples + (uint64_t)g.split_off * kSamplesPerTile;
    const K *As = smp + geo.pb / S;
    const K *Bs = As + W / S;
    const uint64_t d = geo.d0, nA = geo.lenA, nB = geo.lenB;
    uint64_t lo = d > nB ? d - nB : 0;
    uint64_t hi = d < nA ? d : nA;
    if (!active) lo = hi = 0;
    // coarse: first u in [1, hi / S] without Q(u)
    const uint64_t f = group_first_false(1, active ? hi / S + 1 : 1, [&](uint64_t u) {
        return d - u * S >= nB || !O::lt(ldg(Bs + (d - u * S) / S), ldg(As + u - 1));
    });
    const uint64_t u1 = f - 1;
    const uint64_t wl = u1 >= 1 ? max(lo, (u1 - 1) * S + 1) : lo;
    const uint64_t wh = min(hi, (u1 + 1) * S - 1);
    // fine: the first i in [wl, wh) with A[i] > B[d - 1 - i], else wh
    const uint64_t c = group_first_false(wl, wh, [&](uint64_t i) {
        return !O::lt(O::ord(ldg(B + d - 1 - i)), O::ord(ldg(A + i)));
    });
    if (active && gid % kSplitLanes == 0 && half == 0) splits[g.split_off + tile] = (uint32_t)c;
    if constexpr (BOUNDS) {
        // the element at output d of the pair (d < nA + nB for a tile)
        K x = 0;
        if (active) {
            const bool fromA =
                c < nA && (d - c >= nB || !O::lt(O::ord(ldg(B + (d - c))), O::ord(ldg(A + c))));
            x = O::ord(ldg(fromA ? A + c : B + (d - c)));
        }
        const Merge4Geom g4 = merge4_geom(g.m, W, tile);
        // this group's run of the other pair
        const uint32_t r = (g4.which == 0 ? 2 : 0) + half;
        const uint64_t off = g4.gb + r * W;
        const uint64_t cnt = group_count_before<O>((const K *)rg.sk + off,
                                                   smp + off / S,
                                                   active ? g4.n[r] : 0, x, g4.which == 0);
        if (active && gid % kSplitLanes == 0) {
            uint32_t *bd = bounds + 4 * ((uint64_t)g.split_off + tile);
            bd[r] = (uint32_t)cnt;
            if (half == 0) {
                const uint32_t o = g4.which == 0 ? 0 : 2;
                bd[o] = (uint32_t)c;
                bd[o + 1] = (uint32_t)(d - c);
            }
        }
    }
}
// Items: threads, kSplitLanes (two groups for BOUNDS) per tile; `first` is
// a thread index (a multiple of kBlock).  Every lane of a wave takes part in
// each search (lanes past the last tile with empty ranges), so the
// iterations are uniform per workgroup.
template <class O, bool PAIRS, bool BOUNDS, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_merge_split(TaskRef<SortSeg> tasks, uint32_t first,
                                                        uint32_t level, uint32_t step,
                                                        uint32_t total, uint32_t *splits,
                                                        typename O::K *samples0,
                                                        typename O::K *samples1,
                                                        uint32_t *bounds) {
    constexpr uint32_t GPT = BOUNDS ? 2 : 1;
    const uint32_t W = work_total(tasks, total);
    if (W == 0) return;
    const uint64_t lanes = (uint64_t)W * GPT * kSplitLanes;
    uint64_t base = (uint64_t)first + (uint64_t)blockIdx.x * kBlock;
    if constexpr (!LOOP) {
        if (base < lanes)
            merge_split_item<O, PAIRS, BOUNDS>(tasks, (uint32_t)base + threadIdx.x, W, level, step,
                                               splits, samples0, samples1, bounds);
    } else {
        for (; base < lanes; base += (uint64_t)gridDim.x * kBlock)
            merge_split_item<O, PAIRS, BOUNDS>(tasks, (uint32_t)base + threadIdx.x, W, level, step,
                                               splits, samples0, samples1, bounds);
    }
}


// ---- 4-way pass ----------------------------------------------------------------
// Tiles of a 4-way pass run from one boundary to the next in merge order
// (boundaries of both pairs together).  Boundaries of one pair lie at least
// kMergeTile apart in merge order, so two boundaries of different pairs can
// fall close together and leave a tiny tile between them; a workgroup for a
// tile of a hundred elements costs as long as a full one in everything but
// bandwidth.  A tiny tile (fewer than kMerge4Absorb outputs, not the first
// of its group, not the last) is absorbed by the tile before it, which
// cannot be tiny itself (three boundaries within 2 kMerge4Absorb <
// kMergeTile would put two of one pair closer than kMergeTile); a tile then
// holds at most kMergeTile + kMerge4Absorb elements of each pair.
constexpr uint32_t kMerge4Absorb = 256;

// The boundary after the one at tile t (start vector v): the next boundary
// of its own pair or the first boundary of the other pair placed at or after
// it, whichever comes first in merge order; tile = -1 for the end of the
// group (then vec holds the run lengths).
struct Merge4Bnd {
    uint32_t vec[4];
    uint64_t pos;
    int64_t tile;
};
__device__ __forceinline__ Merge4Bnd next_boundary(const uint32_t *bd, uint64_t m, uint64_t W,
                                                   uint64_t t, const uint32_t (&v)[4]) {
    constexpr uint32_t S = kMergeTile;
    const Merge4Geom geo = merge4_geom(m, W, t);
    Merge4Bnd r;
    r.tile = -1;
    r.pos = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        r.vec[q] = geo.n[q];
        r.pos += geo.n[q];
    }
    const uint32_t nP[2] = {geo.n[0] + geo.n[1], geo.n[2] + geo.n[3]};
    const uint64_t first[2] = {geo.gb / S, (geo.gb + 2 * W) / S};  // first tile of each pair
    auto consider = [&](uint64_t c) {
        uint32_t u[4];
        uint64_t pos = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u[q] = bd[4 * c + q];
            pos += u[q];
        }
        if (pos < r.pos) {
            r.pos = pos;
            r.tile = (int64_t)c;
#pragma unroll
            for (int q = 0; q < 4; ++q) r.vec[q] = u[q];
        }
    };
    if ((geo.k + 1) * S < nP[geo.which]) consider(t + 1);
    const uint32_t other = 1 - geo.which;
    const uint32_t placed = other == 0 ? v[0] + v[1] : v[2] + v[3];
    const uint32_t j = (placed + S - 1) / S;
    if ((uint64_t)j * S < nP[other]) consider(first[other] + j);
    return r;
}

// Start and end vector of every 4-way tile, 8 words at the tile's index
// (running the merge workgroups in output order instead was measured slower:
// the concurrent workgroups then crowd a narrow address range).  An absorbed
// tile gets an empty range.  One thread per tile.
__device__ __forceinline__ void merge4_ends_item(TaskRef<SortSeg> tasks, uint32_t w,
                                                 uint32_t level_arg, uint32_t step,
                                                 const uint32_t *bounds, uint32_t *ends) {
    uint32_t tile, a;
    const SortSeg g = task_of(tasks, w, &tile, &a);
    const uint32_t level = task_level(g, level_arg, step);
    const uint64_t W = (uint64_t)g.w0 << level;
    const uint32_t *bd = bounds + 4 * (uint64_t)g.split_off;
    uint32_t s[4];
    uint64_t pos = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        s[r] = bd[4 * tile + r];
        pos += s[r];
    }
    // tiny tiles with a real boundary after them and a tile before them
    auto tiny = [&](uint64_t p0, const Merge4Bnd &nx) {
        return p0 > 0 && nx.tile >= 0 && nx.pos - p0 < kMerge4Absorb;
    };
    const Merge4Bnd n1 = next_boundary(bd, g.m, W, tile, s);
    uint32_t e[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) e[r] = n1.vec[r];
    if (tiny(pos, n1)) {
#pragma unroll
        for (int r = 0; r < 4; ++r) e[r] = s[r];  // absorbed by the tile before
    } else if (n1.tile >= 0) {
        const Merge4Bnd n2 = next_boundary(bd, g.m, W, (uint64_t)n1.tile, n1.vec);
        if (tiny(n1.pos, n2)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) e[r] = n2.vec[r];  // absorbs the tiny tile after
        }
    }
    uint32_t *out = ends + 8 * ((uint64_t)g.split_off + tile);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        out[r] = s[r];
        out[4 + r] = e[r];
    }
}
template <bool LOOP>
__global__ __launch_bounds__(kBlock) void k_merge4_ends(TaskRef<SortSeg> tasks, uint32_t first,
                                                        uint32_t level, uint32_t step,
                                                        uint32_t total, const uint32_t *bounds,
                                                        uint32_t *ends) {
    // items: threads (no barriers)
    const uint32_t W = work_total(tasks, total);
    const uint32_t w0 = first + blockIdx.x * kBlock + threadIdx.x;
    if constexpr (!LOOP) {
        if (w0 < W) merge4_ends_item(tasks, w0, level, step, bounds, ends);
    } else {
        for (uint32_t w = w0; w < W; w += gridDim.x * kBlock)
            merge4_ends_item(tasks, w, level, step, bounds, ends);
    }
}


// Outputs [d, d + N) of the stable merge of X = sk[x0, x0 + nx) and
// Y = sk[y0, y0 + ny) into out[] (X first on ties), d < nx + ny.  The word
// after Y, sk[y0 + ny], holds the largest key 0xffffffff: once Y is used up
// every X element compares <= it, so a step tests only for the end of X
// (X[nx] is read, never taken).  Outputs past nx + ny are garbage (the
// caller stores none of them) and read at most N - 1 words past the
// sentinel.  A step is two LDS reads at addresses one add from i, a compare
// and a select.
// With `from`, also the LDS index each output was read from (to carry
// payloads along).  With HI the elements are 64-bit key/payload words and
// only their upper halves (the keys) are compared.
template <class O, bool HI, class T>
__device__ __forceinline__ bool lds_le(T a, T b) {
    if constexpr (HI) {
        return !O::lt((uint32_t)(b >> 32), (uint32_t)(a >> 32));
    } else {
        return !O::lt(b, a);
    }
}
template <class O, int N, bool FROM = false, class T = uint32_t, bool HI = false>
__device__ __forceinline__ void merge_lds(const T *sk, uint32_t x0, uint32_t nx, uint32_t y0,
                                          uint32_t ny, uint32_t d, T (&out)[N],
                                          uint32_t *from = nullptr) {
    const T *X = sk + x0, *Y = sk + y0;
    uint32_t lo = d > ny ? d - ny : 0, hi = d < nx ? d : nx;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (lds_le<O, HI>(X[mid], Y[d - 1 - mid])) lo = mid + 1;
        else hi = mid;
    }
    uint32_t i = lo;
    const T *Yd = Y + d;  // Y[j] for j = d + q - i
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const T kx = X[i], ky = Yd[q - (int)i];
        const bool takeX = i < nx && lds_le<O, HI>(kx, ky);
        out[q] = takeX ? kx : ky;
        if constexpr (FROM) from[q] = takeX ? x0 + i : y0 + d + q - i;
        i += takeX;
    }
}

// LDS layout of a 4-way tile: A | B | max | C | D | max, i.e. tile element el
// at sk[el + (el >= c2)], with the sentinels merge_lds needs after B (at c2)
// and after D (at cnt + 1); kMerge4Slack words past them take the reads of
// threads whose outputs run past the end.
//
// Outputs per thread of the pair merges and of the final merge: odd counts
// (one more than the power of two that covers the tile) put the lanes'
// diagonals on distinct LDS banks; even ones stack them on a few.
#ifndef QMS_MERGE_ODD
#define QMS_MERGE_ODD 1
#endif
constexpr int kMergeOdd = QMS_MERGE_ODD;
// elements of one pair in a 4-way tile (with an absorbed tiny tile), and the
// outputs per thread that cover them: the pair merges run on half the
// workgroup, the final merge on all of it (odd, see above)
constexpr uint32_t kMerge4Pair = kMergeTile + kMerge4Absorb;
constexpr int kMerge4NBig = (int)((kMerge4Pair + 127) / 128) | kMergeOdd;
constexpr int kMerge4Slack = kMerge4NBig + 1;

// The two pair merges of a 4-way tile in place: A with B by the first half of
// the threads, C with D by the second half, N outputs per thread.  LDS
// elements of type L: the keys, or for key/payload pairs 64-bit words with
// the key in the upper half (HI), so that a payload moves with its key.
constexpr uint32_t kMerge4Lds = 2 * kMerge4Pair + 2 + kMerge4Slack;  // elements of the LDS tile
template <class O, int N, int NT, bool HI, class L>
__device__ __forceinline__ void merge4_halves(L *sk, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t cnt, uint32_t tid) {
    const bool cd = tid >= NT / 2;
    const uint32_t d = (cd ? tid - NT / 2 : tid) * N;
    const uint32_t base = cd ? c2 + 1 : 0, nx = cd ? c3 - c2 : c1, n = cd ? cnt - c2 : c2;
    L o[N];
    if (d < n) merge_lds<O, N, false, L, HI>(sk, base, nx, base + nx, n - nx, d, o);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (d + q < n) sk[base + d + q] = o[q];
    __syncthreads();
}
// The merged pairs sk[0, c2) and sk[c2 + 1, cnt + 1) merged into sk[0, cnt),
// N outputs per thread.
template <class O, int N, bool HI, class L>
__device__ __forceinline__ void merge4_final(L *sk, uint32_t c2, uint32_t cnt, uint32_t tid) {
    L o[N];
    const uint32_t d = tid * N;
    if (d < cnt) merge_lds<O, N, false, L, HI>(sk, 0, c2, c2 + 1, cnt - c2, d, o);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (d + q < cnt) sk[d + q] = o[q];
    __syncthreads();
}

// One workgroup per boundary: the tile from its start vector to its end
// vector (empty for an absorbed tile).  The slices A|B|C|D are staged in
// LDS; A with B and C with D are merged and written back over their own
// slices, then the two halves are merged the same way; about 18 KB of LDS
// and few registers, so that eight workgroups (as many elements in flight
// as the 2-way pass) stay resident per CU.  Key/payload pairs are packed into
// 64-bit LDS words (key above payload) and 64-bit keys take 64-bit words:
// twice the LDS, four workgroups per CU.
#ifndef QMS_MERGE4_WPE
#define QMS_MERGE4_WPE 8
#endif
constexpr int kMerge4Threads = 256;
template <class O, bool PAIRS>
using Merge4Elem = std::conditional_t<PAIRS, uint64_t, typename O::K>;  // LDS element
template <class O, bool PAIRS>
__device__ __forceinline__ void merge4_item(TaskRef<SortSeg> tasks, uint32_t item,
                                            uint32_t level_arg, uint32_t step,
                                            const uint32_t *bounds, const uint32_t *ends,
                                            typename O::K *samples0, typename O::K *samples1,
                                            Merge4Elem<O, PAIRS> *sk) {
    using K = typename O::K;
    static_assert(!PAIRS || sizeof(K) == 4, "pairs carry 32-bit keys");
    using L = Merge4Elem<O, PAIRS>;
    constexpr uint32_t S = kMergeTile;
    constexpr uint32_t SP = kMerge4Pair;  // elements of one pair at most
    constexpr int NT = kMerge4Threads;
    // the key of an LDS element
    auto lkey = [](L x) -> K {
        if constexpr (PAIRS) {
            return (K)(x >> 32);
        } else {
            return x;
        }
    };
    uint32_t tile, a;
    const SortSeg g = task_of(tasks, item, &tile, &a);
    if (tile * (uint64_t)S >= g.m) return;
    const uint32_t level = task_level(g, level_arg, step);
    K *smp_out = samples_out<K>(g, level, samples0, samples1);
    const Regions rg = level_regions(g, level);
    const uint64_t W = (uint64_t)g.w0 << level;
    const Merge4Geom geo = merge4_geom(g.m, W, tile);
    // the tile's start and end vectors
    const uint64_t at = 8 * ((uint64_t)g.split_off + tile);
    uint32_t s[4], len[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        // clamped to the runs and the LDS tile (a no-op for consistent bounds)
        s[r] = min(ends[at + r], geo.n[r]);
        len[r] = min(max(ends[at + 4 + r], s[r]), geo.n[r]) - s[r];
    }
    len[1] = min(len[1], SP - min(len[0], SP));
    len[0] = min(len[0], SP);
    len[3] = min(len[3], SP - min(len[2], SP));
    len[2] = min(len[2], SP);
    const uint32_t c1 = len[0], c2 = c1 + len[1], c3 = c2 + len[2], cnt = c3 + len[3];
    if (cnt == 0) return;
    const uint64_t ps = (uint64_t)s[0] + s[1] + s[2] + s[3];
    K *S_ = (K *)rg.sk + geo.gb;
    const K *T_ = (const K *)rg.dk + geo.gb + ps;
    uint32_t *SV_ = PAIRS ? rg.sv + geo.gb : nullptr;
    const uint32_t *TV_ = PAIRS ? rg.dv + geo.gb + ps : nullptr;
    const uint32_t tid = threadIdx.x;
    // tile element el sits in run r at offset cell(el) from the group base
    // (< 4 W <= m < 2^32); the steps between the runs' offsets are added by
    // comparison (a select chain here is turned into a table in scratch)
    const uint32_t W32 = (uint32_t)W;
    const uint32_t off0 = s[0], d1 = W32 + s[1] - c1 - off0, d2 = W32 + s[2] - (c2 - c1) - s[1],
                   d3 = W32 + s[3] - (c3 - c2) - s[2];
    auto cell = [=](uint32_t el) -> uint32_t {
        return off0 + el + (uint32_t)(el >= c1) * d1 + (uint32_t)(el >= c2) * d2 +
               (uint32_t)(el >= c3) * d3;
    };
    {
        // every load of the tile in flight together (up to 2 SP / NT per
        // thread, as many as the tile needs); the window's buffer element
        // takes its run cell at once (each cell is read and written by the
        // same thread), so no registers hold buffer elements through the merge
        constexpr int Q = (2 * SP + NT - 1) / NT;
        K v[Q], old[Q];
        uint32_t pv[PAIRS ? Q : 1], pold[PAIRS ? Q : 1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if ((uint32_t)q * NT < cnt) {
                const uint32_t el = min((uint32_t)q * NT + tid, cnt - 1);
                v[q] = ldg(S_ + cell(el));
                old[q] = ldg(T_ + el);
                if constexpr (PAIRS) {
                    pv[q] = ldg(SV_ + cell(el));
                    pold[q] = ldg(TV_ + el);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t el = (uint32_t)q * NT + tid;
            if (el < cnt) {
                if constexpr (PAIRS) {
                    sk[el + (el >= c2)] = ((uint64_t)O::ord(v[q]) << 32) | pv[q];
                    stg(SV_ + cell(el), pold[q]);
                } else {
                    sk[el + (el >= c2)] = O::ord(v[q]);
                }
                stg(S_ + cell(el), old[q]);
            }
        }
        if (tid == 0) {  // the largest key (for pairs in the compared upper half)
            sk[c2] = PAIRS ? ~L(0) : (L)key_max<K>();
            sk[cnt + 1] = PAIRS ? ~L(0) : (L)key_max<K>();
        }
    }
    __syncthreads();
    // the merges, with as many outputs per thread as the tile needs (a
    // typical tile holds kMergeTile elements, under half the maximum)
    static_assert((uint32_t)kMerge4NBig * (NT / 2) >= SP && (uint32_t)kMerge4NBig * NT >= 2 * SP,
                  "outputs per thread cover the largest tile");
    if (c2 <= S / 2 && cnt - c2 <= S / 2)
        merge4_halves<O, 2 * S / NT / 2 + kMergeOdd, NT, PAIRS>(sk, c1, c2, c3, cnt, tid);
    else
        merge4_halves<O, kMerge4NBig, NT, PAIRS>(sk, c1, c2, c3, cnt, tid);
    if (cnt <= S)
        merge4_final<O, S / NT + kMergeOdd, PAIRS>(sk, c2, cnt, tid);
    else
        merge4_final<O, kMerge4NBig, PAIRS>(sk, c2, cnt, tid);
    // samples of the output runs: every kSampleStride-th position of the group
    {
        constexpr uint32_t SS = kSampleStride;
        static_assert((2 * SP + SS - 1) / SS + 1 <= (uint32_t)NT, "one sample per thread");
        const uint32_t first = (uint32_t)((SS - ps % SS) % SS);
        const uint32_t el = first + tid * SS;
        if (el < cnt)
            stg(smp_out + (uint64_t)g.split_off * kSamplesPerTile + (geo.gb + ps + el) / SS,
                lkey(sk[el]));
    }
    K *Tw = (K *)rg.dk + geo.gb + ps;
    uint32_t *TVw = PAIRS ? rg.dv + geo.gb + ps : nullptr;
#pragma unroll
    for (int q = 0; q < (int)((2 * SP + NT - 1) / NT); ++q) {
        const uint32_t el = q * NT + tid;
        if (el < cnt) {
            const L x = sk[el];
            stg(Tw + el, O::unord(lkey(x)));
            if constexpr (PAIRS) stg(TVw + el, (uint32_t)x);
        }
    }
}
template <class O, bool PAIRS, bool LOOP>
__global__ __launch_bounds__(kMerge4Threads)
__attribute__((amdgpu_waves_per_eu((PAIRS || sizeof(typename O::K) == 8) ? 4 : QMS_MERGE4_WPE,
                                   (PAIRS || sizeof(typename O::K) == 8) ? 4 : QMS_MERGE4_WPE)))
void k_merge4(TaskRef<SortSeg> tasks, uint32_t first, uint32_t level, uint32_t step,
              const uint32_t *bounds, const uint32_t *ends, typename O::K *samples0,
              typename O::K *samples1) {
    __shared__ Merge4Elem<O, PAIRS> sk_mem[kMerge4Lds];
    Merge4Elem<O, PAIRS> *sk = sk_mem;
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) merge4_item<O, PAIRS>(tasks, item, level, step, bounds, ends, samples0, samples1, sk);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            merge4_item<O, PAIRS>(tasks, item, level, step, bounds, ends, samples0, samples1, sk);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}


template <class O, bool PAIRS>
__device__ __forceinline__ void merge_block(typename O::K *S, uint32_t *SV, typename O::K *D,
                                            uint32_t *DV, uint64_t m, uint64_t W,
                                            uint64_t tile, const uint32_t *splits,
                                            typename O::K *samples_out) {
    using K = typename O::K;
    // the two run slices back to back, then the sentinel merge_lds needs
    // (at cnt) and slack for the reads of threads whose outputs run past cnt
    __shared__ K sk[kMergeTile + 1 + kMerge4Slack];
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
    K oldk[kMergePerThread];
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
    K nk[kMergePerThread];
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
    if (tid == 0) sk[cnt] = key_max<K>();
    __syncthreads();

    // each thread merges NM consecutive outputs of the tile (one more than
    // the tile needs: an odd count keeps the lanes' diagonals on distinct
    // LDS banks)
    constexpr int NM = kMergePerThread + kMergeOdd;
    K ok[NM];
    uint32_t from[PAIRS ? NM : 1];
    uint32_t ov[PAIRS ? NM : 1];
    const uint32_t diag = tid * NM;
    if (diag < cnt) {
        merge_lds<O, NM, PAIRS, K>(sk, 0, na, na, nb, diag, ok, from);
        if constexpr (PAIRS) {
#pragma unroll
            for (int q = 0; q < NM; ++q) ov[q] = sv[min(from[q], cnt - 1)];
        }
    }
    __syncthreads();
    if (diag < cnt) {
#pragma unroll
        for (int q = 0; q < NM; ++q) {
            if (diag + q < cnt) {
                sk[diag + q] = ok[q];
                if constexpr (PAIRS) sv[diag + q] = ov[q];
            }
        }
    }
    __syncthreads();
    // the tile's samples for the next level's split search
    if (tid < kSamplesPerTile && tid * kSampleStride < cnt)
        stg(samples_out + tile * kSamplesPerTile + tid, sk[tid * kSampleStride]);
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
__device__ __forceinline__ void merge2_item(TaskRef<SortSeg> tasks, uint32_t item,
                                            uint32_t level_arg, uint32_t step,
                                            const uint32_t *splits, typename O::K *samples0,
                                            typename O::K *samples1) {
    using K = typename O::K;
    uint32_t tile, a;
    const SortSeg g = task_of(tasks, item, &tile, &a);
    if (tile * (uint64_t)kMergeTile >= g.m) return;
    const uint32_t level = task_level(g, level_arg, step);
    const Regions rg = level_regions(g, level);
    merge_block<O, PAIRS>((K *)rg.sk, PAIRS ? rg.sv : nullptr, (K *)rg.dk,
                          PAIRS ? rg.dv : nullptr, g.m, (uint64_t)g.w0 << level, tile,
                          splits + g.split_off,
                          samples_out<K>(g, level, samples0, samples1) +
                              (uint64_t)g.split_off * kSamplesPerTile);
}
template <class O, bool PAIRS, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_merge(TaskRef<SortSeg> tasks, uint32_t first,
                                                  uint32_t level_arg, uint32_t step,
                                                  const uint32_t *splits, typename O::K *samples0,
                                                  typename O::K *samples1) {
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) merge2_item<O, PAIRS>(tasks, item, level_arg, step, splits, samples0, samples1);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            merge2_item<O, PAIRS>(tasks, item, level_arg, step, splits, samples0, samples1);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}

// One pass: the split search, (4-way) the tile ends, then the merge.
// Host-sized: one workgroup per item.  Device-sized (M.overflow > 0): grids
// from the estimate M.tiles, each kernel followed by an overflow launch of
// M.overflow looping workgroups from where the estimate ends (every split
// launch before the merge launches, which read the splits of neighbouring
// tiles).
template <class O, bool PAIRS>
static hipError_t merge_t(const MergeLaunch &M, const Workspace &ws, hipStream_t st) {
    using K = typename O::K;
    if (M.tiles == 0 && M.overflow == 0) return hipSuccess;
    constexpr bool kFour = !PAIRS || sizeof(K) == 4;  // 4-way passes: payloads with 32-bit keys
    if (M.four_way && !kFour) return hipErrorInvalidValue;
    K *s0 = (K *)ws.samples[0], *s1 = (K *)ws.samples[1];
    const uint32_t T = M.tiles, OV = M.overflow;
    const uint32_t GPT = M.four_way ? 2 : 1;
    // the estimate's launches (none for an estimate of zero tiles), then the
    // looping ones from where the estimate ends: the split's items are
    // threads, the ends' tiles
    const uint32_t sgrid = (uint32_t)(((uint64_t)T * GPT * kSplitLanes + kBlock - 1) / kBlock);
    const uint32_t s_ov = sgrid * kBlock;  // first thread of the split overflow
    const uint32_t egrid = (T + kBlock - 1) / kBlock;
    const uint32_t e_ov = egrid * kBlock;  // first tile of the ends overflow
    {
        ProfScope prof(st, K_MERGE_SPLIT, 0.0);
        if (!M.four_way) {
            if (sgrid)
                hipLaunchKernelGGL((k_merge_split<O, PAIRS, false, false>), dim3(sgrid),
                                   dim3(kBlock), 0, st, M.tasks, 0u, M.level, M.step, T,
                                   ws.splits, s0, s1, (uint32_t *)nullptr);
            if (OV)
                hipLaunchKernelGGL((k_merge_split<O, PAIRS, false, true>), dim3(OV), dim3(kBlock),
                                   0, st, M.tasks, s_ov, M.level, M.step, T, ws.splits, s0, s1,
                                   (uint32_t *)nullptr);
        } else if constexpr (kFour) {
            if (sgrid)
                hipLaunchKernelGGL((k_merge_split<O, false, true, false>), dim3(sgrid),
                                   dim3(kBlock), 0, st, M.tasks, 0u, M.level, M.step, T,
                                   ws.splits, s0, s1, ws.bounds);
            if (OV)
                hipLaunchKernelGGL((k_merge_split<O, false, true, true>), dim3(OV), dim3(kBlock), 0,
                                   st, M.tasks, s_ov, M.level, M.step, T, ws.splits, s0, s1,
                                   ws.bounds);
            if (egrid)
                hipLaunchKernelGGL(k_merge4_ends<false>, dim3(egrid), dim3(kBlock), 0, st, M.tasks,
                                   0u, M.level, M.step, T, (const uint32_t *)ws.bounds, ws.ends);
            if (OV)
                hipLaunchKernelGGL(k_merge4_ends<true>, dim3(OV), dim3(kBlock), 0, st, M.tasks,
                                   e_ov, M.level, M.step, T, (const uint32_t *)ws.bounds, ws.ends);
        }
    }
    {
        // per element: read the run cell and the window cell, write both (a
        // 4-way pass moves each element once for two levels)
        ProfScope prof(st, K_MERGE, M.bytes, M.step ? -1 : (int)M.level);
        if (!M.four_way) {
            if (T)
                hipLaunchKernelGGL((k_merge<O, PAIRS, false>), dim3(T), dim3(kBlock), 0, st,
                                   M.tasks, 0u, M.level, M.step, (const uint32_t *)ws.splits, s0,
                                   s1);
            if (OV)
                hipLaunchKernelGGL((k_merge<O, PAIRS, true>), dim3(OV), dim3(kBlock), 0, st,
                                   M.tasks, T, M.level, M.step, (const uint32_t *)ws.splits, s0, s1);
        } else if constexpr (kFour) {
            if (T)
                hipLaunchKernelGGL((k_merge4<O, PAIRS, false>), dim3(T), dim3(kMerge4Threads), 0,
                                   st, M.tasks, 0u, M.level, M.step, (const uint32_t *)ws.bounds,
                                   (const uint32_t *)ws.ends, s0, s1);
            if (OV)
                hipLaunchKernelGGL((k_merge4<O, PAIRS, true>), dim3(OV), dim3(kMerge4Threads), 0,
                                   st, M.tasks, T, M.level, M.step, (const uint32_t *)ws.bounds,
                                   (const uint32_t *)ws.ends, s0, s1);
        }
    }
    return hipGetLastError();
}

hipError_t launch_merge_pass(int dt, bool pairs, const MergeLaunch &M, const Workspace &ws,
                             hipStream_t st) {
    switch (dt) {
    case 0:
        return pairs ? merge_t<OrdU32, true>(M, ws, st) : merge_t<OrdU32, false>(M, ws, st);
    case 1:
        return pairs ? merge_t<OrdF32, true>(M, ws, st) : merge_t<OrdF32, false>(M, ws, st);
    case 2:  // 64-bit keys (with payloads: 2-way passes only)
        return pairs ? merge_t<OrdU64, true>(M, ws, st) : merge_t<OrdU64, false>(M, ws, st);
    case 3:
        return pairs ? merge_t<OrdF64, true>(M, ws, st) : merge_t<OrdF64, false>(M, ws, st);
    case 4:  // uint32 keys in log order (keys only)
        return pairs ? hipErrorInvalidValue : merge_t<OrdLogU32, false>(M, ws, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace qms
