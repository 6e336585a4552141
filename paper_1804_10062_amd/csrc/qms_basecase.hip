// qms_basecase.hip -- the base case X of QuickMergeXsort on gfx950.
//
// Sec. "QuickMergeXsort": below a size threshold Mergesort hands a block to a
// sorting algorithm X and then moves the sorted block to the place Mergesort
// expects it.  Here X is a bitonic sorting network run by one workgroup on a
// tile of up to kBaseTile keys staged in LDS, with the 16 keys a thread owns
// sorted in registers.  Two modes:
//   in place  -- the sorted tile is written back where it was read;
//   swap      -- the sorted tile is written into the buffer region and the
//                buffer elements found there move into the vacated source
//                cells (the swap-instead-of-move principle of Sec.
//                "QuickXsort and QuickMergesort"; Fig. 2's msort base case).
// Short tiles are padded with the largest key; for key/payload pairs each
// LDS entry is (key << 32 | index), so padding sorts after real keys and the
// payload is gathered through the index.
#include <type_traits>

#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

namespace qms {

// padded LDS index: one spare word every 16 words breaks the 16-way bank
// conflicts of the per-thread runs of 16 consecutive entries
__device__ __forceinline__ uint32_t lds_idx(uint32_t i) { return i + (i >> 4); }

template <class E>
__device__ __forceinline__ void cmpx(E &a, E &b, bool asc) {
    E lo = a < b ? a : b;
    E hi = a < b ? b : a;
    a = asc ? lo : hi;
    b = asc ? hi : lo;
}

template <bool PAIRS>
struct TileElem;
template <>
struct TileElem<false> {
    using E = uint32_t;
    __device__ static E make(uint32_t k, uint32_t) { return k; }
    __device__ static E pad(uint32_t) { return 0xFFFFFFFFu; }
    __device__ static uint32_t key(E x) { return x; }
    __device__ static uint32_t index(E) { return 0; }
};
template <>
struct TileElem<true> {
    using E = uint64_t;
    __device__ static E make(uint32_t k, uint32_t i) { return ((uint64_t)k << 32) | i; }
    __device__ static E pad(uint32_t i) { return (0xFFFFFFFFull << 32) | i; }
    __device__ static uint32_t key(E x) { return (uint32_t)(x >> 32); }
    __device__ static uint32_t index(E x) { return (uint32_t)x; }
};

// Sort one tile.  src/dst are the tile's first cells in the source and the
// destination region (equal in place), len <= kBaseTile.
template <class O, bool PAIRS>
__device__ __forceinline__ void tile_sort_block(uint32_t *sk, uint32_t *sv, uint32_t *dk,
                                                uint32_t *dv, uint32_t len, bool swap) {
    using TE = TileElem<PAIRS>;
    using E = typename TE::E;
    __shared__ E s[kBaseTile + kBaseTile / 16];
    __shared__ uint32_t sp[PAIRS ? kBaseTile : 1];
    const uint32_t tid = threadIdx.x;

    uint32_t oldk[kBasePerThread];
    uint32_t oldv[PAIRS ? kBasePerThread : 1];
#pragma unroll
    for (int q = 0; q < kBasePerThread; ++q) {
        const uint32_t e = q * kBlock + tid;
        E x;
        if (e < len) {
            x = TE::make(O::ord(sk[e]), e);
            if constexpr (PAIRS) sp[e] = sv[e];
            if (swap) {
                oldk[q] = dk[e];
                if constexpr (PAIRS) oldv[q] = dv[e];
            }
        } else {
            x = TE::pad(e);
        }
        s[lds_idx(e)] = x;
    }
    __syncthreads();

    E r[kBasePerThread];
    const uint32_t base = tid * kBasePerThread;
#pragma unroll
    for (int i = 0; i < kBasePerThread; ++i) r[i] = s[lds_idx(base + i)];
    // runs of 16 in registers, alternating direction (bitonic stages k <= 16)
#pragma unroll
    for (int k = 2; k <= kBasePerThread; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j >= 1; j >>= 1) {
#pragma unroll
            for (int i = 0; i < kBasePerThread; ++i) {
                const int l = i ^ j;
                if (l > i) cmpx(r[i], r[l], ((base + i) & k) == 0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kBasePerThread; ++i) s[lds_idx(base + i)] = r[i];
    __syncthreads();

    for (uint32_t k = 2 * kBasePerThread; k <= (uint32_t)kBaseTile; k <<= 1) {
        for (uint32_t j = k >> 1; j >= (uint32_t)kBasePerThread; j >>= 1) {
#pragma unroll
            for (int q = 0; q < kBaseTile / 2 / kBlock; ++q) {
                const uint32_t p = q * kBlock + tid;
                const uint32_t i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                const uint32_t l = i | j;
                E a = s[lds_idx(i)], b = s[lds_idx(l)];
                cmpx(a, b, (i & k) == 0);
                s[lds_idx(i)] = a;
                s[lds_idx(l)] = b;
            }
            __syncthreads();
        }
        const bool asc = (base & k) == 0;
#pragma unroll
        for (int i = 0; i < kBasePerThread; ++i) r[i] = s[lds_idx(base + i)];
#pragma unroll
        for (int j = kBasePerThread / 2; j >= 1; j >>= 1) {
#pragma unroll
            for (int i = 0; i < kBasePerThread; ++i) {
                const int l = i ^ j;
                if (l > i) cmpx(r[i], r[l], asc);
            }
        }
#pragma unroll
        for (int i = 0; i < kBasePerThread; ++i) s[lds_idx(base + i)] = r[i];
        __syncthreads();
    }

#pragma unroll
    for (int q = 0; q < kBasePerThread; ++q) {
        const uint32_t e = q * kBlock + tid;
        if (e < len) {
            const E x = s[lds_idx(e)];
            dk[e] = O::unord(TE::key(x));
            if constexpr (PAIRS) dv[e] = sp[TE::index(x)];
            if (swap) {
                sk[e] = oldk[q];
                if constexpr (PAIRS) sv[e] = oldv[q];
            }
        }
    }
}

// One workgroup per base tile of every Mergesort task in the table.
template <class O, bool PAIRS>
__global__ __launch_bounds__(kBlock) void k_tile_sort(TaskRef<SortSeg> tasks) {
    uint32_t t, a;
    const SortSeg g = task_of(tasks, blockIdx.x, &t, &a);
    const uint32_t t0 = t * kBaseTile;
    if (t0 >= g.m) return;
    const uint32_t len = min((uint32_t)kBaseTile, g.m - t0);
    const bool swap = (g.L & 1u) != 0;
    const uint32_t src = g.D + t0, dst = (swap ? g.Bf : g.D) + t0;
    tile_sort_block<O, PAIRS>(g.keys + src, PAIRS ? g.vals + src : nullptr, g.keys + dst,
                              PAIRS ? g.vals + dst : nullptr, len, swap);
}

template <class O, bool PAIRS>
static hipError_t tile_sort_t(const TaskRef<SortSeg> &tasks, uint32_t tiles, double bytes,
                              hipStream_t st) {
    if (tiles == 0) return hipSuccess;
    ProfScope prof(st, K_TILE_SORT, bytes);
    hipLaunchKernelGGL((k_tile_sort<O, PAIRS>), dim3(tiles), dim3(kBlock), 0, st, tasks);
    return hipGetLastError();
}

hipError_t launch_tile_sort(int dt, bool pairs, const TaskRef<SortSeg> &tasks, uint32_t tiles,
                            double bytes, hipStream_t st) {
    if (dt == 1)
        return pairs ? tile_sort_t<OrdF32, true>(tasks, tiles, bytes, st)
                     : tile_sort_t<OrdF32, false>(tasks, tiles, bytes, st);
    return pairs ? tile_sort_t<OrdU32, true>(tasks, tiles, bytes, st)
                 : tile_sort_t<OrdU32, false>(tasks, tiles, bytes, st);
}

}  // namespace qms
