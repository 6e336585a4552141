// qms_bitonic.hip -- the sorting algorithm X that finishes the loop's last
// range, in place, on gfx950.
//
// Sec. "QuickXsort and QuickMergesort" leaves X open: QuickXsort partitions,
// sorts one side with X while the other serves as its buffer, and continues
// on the rest.  The loop here runs until its range holds at most final_tile
// keys and then sorts that range with a bitonic network (QuickMergeXsort's
// idea of handing small blocks to another algorithm, applied once at the
// loop level): every exchange is between two cells of the range, so no
// memory beyond the range is used, and for a range of F keys the network
// adds O(F log^2 F) comparisons to the n lg n + O(n) of the loop, which for
// F << n is a negligible share.
//
// The network is the bitonic merge-sort in its all-ascending form, which
// sorts any length: tiles of the base tile T are sorted first (the base
// case); stage k then merges ascending runs of 2^(k-1) into runs of 2^k by
// comparing position i with i ^ (2^k - 1) (the mirror step) and then i with
// i + j for j = 2^(k-2), ..., 1 (half-cleaners), all ascending.  Positions at
// or beyond the range's end act as +infinity: a pair whose upper position
// lies outside is left alone, so the cells past the range are never read or
// written.  Four kernels share the work of a stage:
//   mirror+columns -- the mirror step and the first (up to four) half-
//                 cleaner steps in one pass: a thread holds a column of the
//                 lower half of a 2^k block (positions that differ only in
//                 the bits of those steps) and the mirrored column of the
//                 upper half, exchanges each lower element with its mirror,
//                 then runs the half-cleaner steps on both columns in
//                 registers;
//   mirror     -- the mirror step alone (the first stage, whose half-cleaner
//                 steps all lie inside the tiles);
//   columns    -- up to four further consecutive half-cleaner steps with
//                 j >= T in one pass: a thread holds the 2, 4, 8 or 16
//                 elements whose positions differ only in those bits and
//                 exchanges them in registers; rows are read and written as
//                 contiguous runs;
//   tile       -- the half-cleaner steps j < T inside each tile of T keys:
//                 the last stage of the base case's network (registers,
//                 lane exchanges and the LDS).
// Several ranges (a batch) share each launch through task tables.
#include <algorithm>

#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

namespace qms {

namespace {

constexpr uint32_t kMirrorPer = kMirrorChunk / kBitThreads;  // mirror pairs per thread

// ---- mirror step of stage k -------------------------------------------------------
// Pair t (t-th position of the lower halves of the 2^k blocks) is position
// i = (t / 2^(k-1)) * 2^k + t % 2^(k-1) and its partner i ^ (2^k - 1).
template <class O, bool PAIRS>
__device__ __forceinline__ void mirror_item(TaskRef<SortSeg> tasks, uint32_t item, uint32_t k) {
    using K = typename O::K;
    uint32_t c, a;
    const SortSeg g = task_of(tasks, item, &c, &a);
    K *keys = (K *)g.keys;
    uint32_t *vals = g.vals;
    const uint64_t m = g.m, H = 1ull << (k - 1), B = 2 * H;
    uint64_t pi[kMirrorPer], pp[kMirrorPer];
    K x[kMirrorPer], y[kMirrorPer];
    bool on[kMirrorPer];
#pragma unroll
    for (uint32_t q = 0; q < kMirrorPer; ++q) {
        const uint64_t t = (uint64_t)c * kMirrorChunk + (uint64_t)q * kBitThreads + threadIdx.x;
        const uint64_t i = (t / H) * B + (t % H);
        const uint64_t p = i ^ (B - 1);
        on[q] = p < m;
        pi[q] = i;
        pp[q] = p;
        if (on[q]) {
            x[q] = ldg(keys + i);
            y[q] = ldg(keys + p);
        }
    }
#pragma unroll
    for (uint32_t q = 0; q < kMirrorPer; ++q) {
        if (!on[q] || !O::lt(O::ord(y[q]), O::ord(x[q]))) continue;
        keys[pi[q]] = y[q];
        keys[pp[q]] = x[q];
        if (PAIRS) {
            const uint32_t u = vals[pi[q]], w = vals[pp[q]];
            vals[pi[q]] = w;
            vals[pp[q]] = u;
        }
    }
}

// Items: one workgroup each (host-sized: the grid is the item count), or
// with tasks.dyn the plan's count, which the workgroups take in grid-stride
// order.
template <class O, bool PAIRS>
__global__ __launch_bounds__(kBitThreads) void k_bitonic_mirror(TaskRef<SortSeg> tasks,
                                                                uint32_t items, uint32_t k) {
    const uint32_t W = work_total(tasks, items);
    for (uint32_t it = blockIdx.x; it < W; it += gridDim.x) mirror_item<O, PAIRS>(tasks, it, k);
}

// ---- half-cleaner steps j = 2^hi, ..., 2^lo (j >= T) ------------------------------
// Blocks of 2^(hi+1) positions; in a block, row r (bits lo..hi) and column
// col (bits below lo): position blk * 2^(hi+1) + r * 2^lo + col.  A thread
// owns one column of one block and its R = 2^(hi-lo+1) rows.
template <class O, bool PAIRS, int R>
__device__ __forceinline__ void columns_item(TaskRef<SortSeg> tasks, uint32_t item, uint32_t lo,
                                             uint32_t hi) {
    using K = typename O::K;
    uint32_t c, a;
    const SortSeg g = task_of(tasks, item, &c, &a);
    K *keys = (K *)g.keys;
    uint32_t *vals = g.vals;
    const uint64_t m = g.m;
    const uint32_t cpb = (1u << lo) / kBitThreads;  // column chunks per block
    const uint64_t blk = c / cpb;
    const uint64_t col = (uint64_t)(c % cpb) * kBitThreads + threadIdx.x;
    const uint64_t base = (blk << (hi + 1)) + col;
    K x[R];
    uint32_t v[R];
    bool on[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t i = base + ((uint64_t)r << lo);
        on[r] = i < m;
        x[r] = on[r] ? O::ord(ldg(keys + i)) : key_max<K>();
        if (PAIRS) v[r] = on[r] ? ldg(vals + i) : 0u;
    }
#pragma unroll
    for (int d = R / 2; d >= 1; d /= 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & d) continue;
            // the upper element outside the range is +infinity: no exchange
            if (on[r + d] && O::lt(x[r + d], x[r])) {
                const K t = x[r];
                x[r] = x[r + d];
                x[r + d] = t;
                if (PAIRS) {
                    const uint32_t u = v[r];
                    v[r] = v[r + d];
                    v[r + d] = u;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!on[r]) continue;
        const uint64_t i = base + ((uint64_t)r << lo);
        keys[i] = O::unord(x[r]);
        if (PAIRS) vals[i] = v[r];
    }
}

template <class O, bool PAIRS, int R>
__global__ __launch_bounds__(kBitThreads) void k_bitonic_columns(TaskRef<SortSeg> tasks,
                                                                 uint32_t items, uint32_t lo,
                                                                 uint32_t hi) {
    const uint32_t W = work_total(tasks, items);
    for (uint32_t it = blockIdx.x; it < W; it += gridDim.x)
        columns_item<O, PAIRS, R>(tasks, it, lo, hi);
}

// ---- mirror step and half-cleaner steps 2^hi .. 2^lo (hi = k - 2) of stage k ---------
// Block blk of 2^k positions: a thread owns column col of its lower half,
// rows r < R (bits lo..k-2; position blk 2^k + r 2^lo + col), and the
// mirrored column 2^lo - 1 - col of its upper half, rows r' < R (position
// blk 2^k + 2^(k-1) + r' 2^lo + 2^lo - 1 - col): the mirror of lower row r is
// upper row R - 1 - r.
template <class O, bool PAIRS, int R>
__device__ __forceinline__ void mirror_columns_item(TaskRef<SortSeg> tasks, uint32_t item,
                                                    uint32_t k, uint32_t lo) {
    using K = typename O::K;
    uint32_t c, a;
    const SortSeg g = task_of(tasks, item, &c, &a);
    K *keys = (K *)g.keys;
    uint32_t *vals = g.vals;
    const uint64_t m = g.m;
    const uint32_t cpb = (1u << lo) / kBitThreads;  // column chunks per block
    const uint64_t blk = c / cpb;
    const uint64_t col = (uint64_t)(c % cpb) * kBitThreads + threadIdx.x;
    const uint64_t baseL = (blk << k) + col;
    const uint64_t baseU = (blk << k) + (1ull << (k - 1)) + ((1ull << lo) - 1 - col);
    K xl[R], xu[R];
    uint32_t vl[R], vu[R];
    bool ol[R], ou[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t i = baseL + ((uint64_t)r << lo);
        const uint64_t j = baseU + ((uint64_t)r << lo);
        ol[r] = i < m;
        ou[r] = j < m;
        xl[r] = ol[r] ? O::ord(ldg(keys + i)) : key_max<K>();
        xu[r] = ou[r] ? O::ord(ldg(keys + j)) : key_max<K>();
        if (PAIRS) {
            vl[r] = ol[r] ? ldg(vals + i) : 0u;
            vu[r] = ou[r] ? ldg(vals + j) : 0u;
        }
    }
    // the mirror step (an upper element outside the range is +infinity)
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = R - 1 - r;
        if (ou[q] && O::lt(xu[q], xl[r])) {
            const K t = xl[r];
            xl[r] = xu[q];
            xu[q] = t;
            if (PAIRS) {
                const uint32_t u = vl[r];
                vl[r] = vu[q];
                vu[q] = u;
            }
        }
    }
    // the half-cleaner steps inside each half
#pragma unroll
    for (int d = R / 2; d >= 1; d /= 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r & d) continue;
            if (ol[r + d] && O::lt(xl[r + d], xl[r])) {
                const K t = xl[r];
                xl[r] = xl[r + d];
                xl[r + d] = t;
                if (PAIRS) {
                    const uint32_t u = vl[r];
                    vl[r] = vl[r + d];
                    vl[r + d] = u;
                }
            }
            if (ou[r + d] && O::lt(xu[r + d], xu[r])) {
                const K t = xu[r];
                xu[r] = xu[r + d];
                xu[r + d] = t;
                if (PAIRS) {
                    const uint32_t u = vu[r];
                    vu[r] = vu[r + d];
                    vu[r + d] = u;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (ol[r]) {
            const uint64_t i = baseL + ((uint64_t)r << lo);
            keys[i] = O::unord(xl[r]);
            if (PAIRS) vals[i] = vl[r];
        }
        if (ou[r]) {
            const uint64_t j = baseU + ((uint64_t)r << lo);
            keys[j] = O::unord(xu[r]);
            if (PAIRS) vals[j] = vu[r];
        }
    }
}

template <class O, bool PAIRS, int R>
__global__ __launch_bounds__(kBitThreads) void k_bitonic_mirror_columns(TaskRef<SortSeg> tasks,
                                                                        uint32_t items,
                                                                        uint32_t k, uint32_t lo) {
    const uint32_t W = work_total(tasks, items);
    for (uint32_t it = blockIdx.x; it < W; it += gridDim.x)
        mirror_columns_item<O, PAIRS, R>(tasks, it, k, lo);
}

template <class O, bool PAIRS>
static hipError_t bitonic_t(int dt, const BitonicLaunch &L, hipStream_t st) {
    if (L.items == 0) return hipSuccess;
    ProfScope prof(st, K_FINAL, L.bytes);
    switch (L.kind) {
    case BitonicLaunch::MIRROR:
        hipLaunchKernelGGL((k_bitonic_mirror<O, PAIRS>), dim3(L.items), dim3(kBitThreads), 0, st,
                           L.tasks, L.items, L.k);
        break;
    case BitonicLaunch::COLUMNS:
        switch (L.hi - L.lo + 1) {
        case 1:
            hipLaunchKernelGGL((k_bitonic_columns<O, PAIRS, 2>), dim3(L.items), dim3(kBitThreads),
                               0, st, L.tasks, L.items, L.lo, L.hi);
            break;
        case 2:
            hipLaunchKernelGGL((k_bitonic_columns<O, PAIRS, 4>), dim3(L.items), dim3(kBitThreads),
                               0, st, L.tasks, L.items, L.lo, L.hi);
            break;
        case 3:
            hipLaunchKernelGGL((k_bitonic_columns<O, PAIRS, 8>), dim3(L.items), dim3(kBitThreads),
                               0, st, L.tasks, L.items, L.lo, L.hi);
            break;
        case 4:
            hipLaunchKernelGGL((k_bitonic_columns<O, PAIRS, 16>), dim3(L.items),
                               dim3(kBitThreads), 0, st, L.tasks, L.items, L.lo, L.hi);
            break;
        default:
            return hipErrorInvalidValue;
        }
        break;
    case BitonicLaunch::MIRROR_COLUMNS:
        switch (L.hi - L.lo + 1) {
        case 1:
            hipLaunchKernelGGL((k_bitonic_mirror_columns<O, PAIRS, 2>), dim3(L.items),
                               dim3(kBitThreads), 0, st, L.tasks, L.items, L.k, L.lo);
            break;
        case 2:
            hipLaunchKernelGGL((k_bitonic_mirror_columns<O, PAIRS, 4>), dim3(L.items),
                               dim3(kBitThreads), 0, st, L.tasks, L.items, L.k, L.lo);
            break;
        case 3:
            hipLaunchKernelGGL((k_bitonic_mirror_columns<O, PAIRS, 8>), dim3(L.items),
                               dim3(kBitThreads), 0, st, L.tasks, L.items, L.k, L.lo);
            break;
        case 4:
            hipLaunchKernelGGL((k_bitonic_mirror_columns<O, PAIRS, 16>), dim3(L.items),
                               dim3(kBitThreads), 0, st, L.tasks, L.items, L.k, L.lo);
            break;
        default:
            return hipErrorInvalidValue;
        }
        break;
    case BitonicLaunch::TILE:
        return launch_tile_merge(dt, PAIRS, L.tasks, L.items, st);
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

std::vector<BitonicLaunch> bitonic_passes(uint32_t K, uint32_t lt) {
    std::vector<BitonicLaunch> v;
    for (uint32_t k = lt + 1; k <= K; ++k) {
        BitonicLaunch L;
        int hi = (int)k - 2;
        L.k = k;
        if (hi < (int)lt) {
            L.kind = BitonicLaunch::MIRROR;  // no half-cleaner step above the tile
        } else {
            L.kind = BitonicLaunch::MIRROR_COLUMNS;
            L.hi = (uint32_t)hi;
            L.lo = (uint32_t)std::max<int>((int)lt, hi - 3);
            hi -= 4;
        }
        v.push_back(L);
        for (; hi >= (int)lt; hi -= 4) {
            L = BitonicLaunch{};
            L.kind = BitonicLaunch::COLUMNS;
            L.k = k;
            L.hi = (uint32_t)hi;
            L.lo = (uint32_t)std::max<int>((int)lt, hi - 3);
            v.push_back(L);
        }
        L = BitonicLaunch{};
        L.kind = BitonicLaunch::TILE;
        L.k = k;
        v.push_back(L);
    }
    return v;
}

hipError_t launch_bitonic_pass(int dt, bool pairs, const BitonicLaunch &L, hipStream_t st) {
    switch (dt) {
    case 0:
        return pairs ? bitonic_t<OrdU32, true>(dt, L, st) : bitonic_t<OrdU32, false>(dt, L, st);
    case 1:
        return pairs ? bitonic_t<OrdF32, true>(dt, L, st) : bitonic_t<OrdF32, false>(dt, L, st);
    case 2:
        return pairs ? bitonic_t<OrdU64, true>(dt, L, st) : bitonic_t<OrdU64, false>(dt, L, st);
    case 3:
        return pairs ? bitonic_t<OrdF64, true>(dt, L, st) : bitonic_t<OrdF64, false>(dt, L, st);
    case 4:
        return pairs ? hipErrorInvalidValue : bitonic_t<OrdLogU32, false>(dt, L, st);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace qms
