// qms_select.hip -- the worst-case pivot of HybridQuickMergesort on gfx950.
//
// Sec. "Worst-Case Efficient QuickMergeSort": after a partition whose pivot
// fell outside [delta n, (1 - delta) n] (delta = 1/16), the next pivot is the
// median of the n/3 medians of three (MoMQuickMergesort's pivot); later
// rounds return to median-of-3.  That pivot has at least 2 floor(n/6) keys
// <= it and as many >= it, so the next split is balanced whatever the input.
//
// The paper finds the median of the medians with the median-of-medians
// selection algorithm; any exact selection gives the same value.  Here it is
// a most-significant-digit radix select over the virtual array of medians
//     M[i] = median(key[3i], key[3i + 1], key[3i + 2]),   i < c = floor(s / 3)
// (order-mapped keys), target rank r = floor((c - 1) / 2) (the lower median):
// one pass per 8-bit digit (four for 32-bit keys, eight for 64-bit), each a
// histogram of the digit among the medians that match the digits chosen so
// far, then a pick of the bucket that holds rank r.  The medians are recomputed from the keys in every pass, so
// no array of n/3 words is ever stored; each pass reads the range once.
//
// All segments that need the pivot in a round are served by the same
// launches (task tables); each has a 256-bin histogram in the workspace.
// The last histogram workgroup of a segment in a pass (a per-segment count
// of finished workgroups) picks the bucket, so a pass is one launch.
#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

namespace qms {


__device__ __forceinline__ const PartSeg &mom_seg(const TaskRef<PartSeg> &r, uint32_t a) {
    return r.A == 1 ? r.one : r.tab[a];
}

// Clear the histogram, set rank and prefix, no histogram workgroup done
// (kBlock threads; also called by the device-side round plan).
__device__ __forceinline__ void mom_init_segment(const PartSeg &g, uint64_t *meta_all,
                                                 uint32_t *hist_all) {
    stg(hist_all + (uint64_t)g.pad * 256 + threadIdx.x, 0u);
    if (threadIdx.x == 0) {
        uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
        const uint64_t c = g.s / 3;
        meta[M_MOM_RANK] = (c - 1) / 2;
        meta[M_MOM_PREFIX] = 0;
        meta[M_MOM_DONE] = 0;
    }
}
// One workgroup per segment.
__global__ __launch_bounds__(kBlock) void k_mom_init(TaskRef<PartSeg> tasks, uint64_t *meta_all,
                                                     uint32_t *hist_all) {
    mom_init_segment(mom_seg(tasks, blockIdx.x), meta_all, hist_all);
}

// The bucket that holds rank r: the prefix grows by its digit and r becomes
// the rank inside it; the histogram is cleared for the next pass.  After the
// last pass the prefix is the pivot.  The histogram was filled by atomics
// of other workgroups: it is read and cleared with agent-scope atomics.
__device__ __forceinline__ void mom_pick_segment(const PartSeg &g, uint32_t pass, uint32_t last,
                                                 uint64_t *meta_all, uint32_t *hist_all,
                                                 uint32_t *tmp) {
    uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
    uint32_t *hist = hist_all + (uint64_t)g.pad * 256;
    const uint32_t b = threadIdx.x;
    const uint32_t v = __hip_atomic_exchange(hist + b, 0u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t r = (uint32_t)meta[M_MOM_RANK];
    const uint64_t prefix = meta[M_MOM_PREFIX];
    uint32_t total;
    const uint32_t below = block_exclusive_scan(v, tmp, &total);  // ends with a barrier
    if (below <= r && r < below + v) {
        const uint64_t np = (prefix << 8) | b;
        meta[M_MOM_RANK] = r - below;
        meta[M_MOM_PREFIX] = np;
        if (pass == last) meta[M_PIVOT] = np;
    }
    if (b == 0)
        __hip_atomic_store(meta + M_MOM_DONE, (uint64_t)0, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Histogram of digit `pass` (the pass-th byte from the top) of the medians
// whose higher digits equal the prefix chosen so far; the segment's last
// workgroup to finish picks the digit.
template <class O>
__device__ __forceinline__ void mom_hist_item(TaskRef<PartSeg> tasks, uint32_t item,
                                              uint32_t pass, uint32_t last, uint64_t *meta_all,
                                              uint32_t *hist_all, uint32_t *h, uint32_t *tmp) {
    using K = typename O::K;
    constexpr uint32_t kBits = 8 * sizeof(K);
    uint32_t t, a;
    const PartSeg g = task_of_wave(tasks, item, &t, &a);
    const K *keys = (const K *)g.keys + g.lo;
    const uint64_t c = g.s / 3;
    const K prefix = (K)meta_all[(uint64_t)g.slot * M_COUNT + M_MOM_PREFIX];
    const uint32_t shift = kBits - 8 - 8 * pass;
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t i0 = (uint64_t)t * kMomTile;
    // clamped, unconditional loads (all in flight), masked afterwards
    K k0[kMomPerThread], k1[kMomPerThread], k2[kMomPerThread];
#pragma unroll
    for (int q = 0; q < kMomPerThread; ++q) {
        uint64_t i = i0 + (uint64_t)q * kBlock + threadIdx.x;
        i = i < c ? i : c - 1;
        k0[q] = ldg(keys + 3 * i);
        k1[q] = ldg(keys + 3 * i + 1);
        k2[q] = ldg(keys + 3 * i + 2);
    }
#pragma unroll
    for (int q = 0; q < kMomPerThread; ++q) {
        const uint64_t i = i0 + (uint64_t)q * kBlock + threadIdx.x;
        const K m = median3(O::ord(k0[q]), O::ord(k1[q]), O::ord(k2[q]));
        // the digits above this one (none in the first pass)
        const bool match = pass == 0 || (m >> (shift + 8 < kBits ? shift + 8 : 0)) == prefix;
        if (i < c && match) atomicAdd(&h[(uint32_t)(m >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t v = h[threadIdx.x];
    // The histogram, the count of finished workgroups and the last
    // workgroup's reads of the histogram are all agent-scope atomics, which
    // every workgroup performs at the same coherent point; ordering them
    // needs only that each add has been performed (its result has come back)
    // before the count goes up.  No fence: an agent-scope fence writes back
    // and invalidates the whole L2 of the workgroup's XCD, which serialises
    // across the workgroups of a launch.
    if (v != 0) {
        const uint32_t old = __hip_atomic_fetch_add(hist_all + (uint64_t)g.pad * 256 + threadIdx.x,
                                                    v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        asm volatile("" ::"v"(old));  // wait for the result
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint64_t done = __hip_atomic_fetch_add(
            meta_all + (uint64_t)g.slot * M_COUNT + M_MOM_DONE, (uint64_t)1, __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT);
        h[0] = done + 1 == mom_tiles_of(g.s) ? 1u : 0u;
    }
    __syncthreads();
    const bool is_last = h[0] != 0;
    __syncthreads();  // h is reused by the next item
    if (is_last) mom_pick_segment(g, pass, last, meta_all, hist_all, tmp);
}
template <class O, bool LOOP>
__global__ __launch_bounds__(kBlock) void k_mom_hist(TaskRef<PartSeg> tasks, uint32_t first,
                                                     uint32_t pass, uint32_t last,
                                                     uint64_t *meta_all, uint32_t *hist_all) {
    __shared__ uint32_t h_mem[256];
    __shared__ uint32_t tmp_mem[kWaves + 1];
    uint32_t *h = h_mem, *tmp = tmp_mem;
    const uint32_t W = work_total(tasks, first + gridDim.x);
    if constexpr (!LOOP) {
        const uint32_t item = first + blockIdx.x;
        if (item < W) mom_hist_item<O>(tasks, item, pass, last, meta_all, hist_all, h, tmp);
    } else {
        for (uint32_t item = first + blockIdx.x; item < W; item += gridDim.x) {
            mom_hist_item<O>(tasks, item, pass, last, meta_all, hist_all, h, tmp);
            __syncthreads();  // the LDS is reused by the next item
        }
    }
}

// init: one workgroup per segment, unless `init` is false (the round plan
// initialised them).  tiles: the histogram workgroups of a host-sized
// launch; with tasks.dyn the estimate of a device-sized one, followed in
// each pass by an overflow launch of `overflow` looping workgroups.
template <class O>
static hipError_t mom_t(const TaskRef<PartSeg> &tasks, uint32_t tiles, uint32_t overflow,
                        bool init, const Workspace &ws, hipStream_t st) {
    ProfScope prof(st, K_PART_SCAN, 0.0);
    constexpr uint32_t kPasses = sizeof(typename O::K);  // 8-bit digits
    if (init)
        hipLaunchKernelGGL(k_mom_init, dim3(tasks.A), dim3(kBlock), 0, st, tasks, ws.meta,
                           ws.hist);
    if (tiles == 0 && overflow == 0) return hipGetLastError();
    for (uint32_t pass = 0; pass < kPasses; ++pass) {
        if (tiles)
            hipLaunchKernelGGL((k_mom_hist<O, false>), dim3(tiles), dim3(kBlock), 0, st, tasks,
                               0u, pass, kPasses - 1, ws.meta, ws.hist);
        if (overflow)
            hipLaunchKernelGGL((k_mom_hist<O, true>), dim3(overflow), dim3(kBlock), 0, st, tasks,
                               tiles, pass, kPasses - 1, ws.meta, ws.hist);
    }
    return hipGetLastError();
}

uint32_t mom_tiles(uint64_t s) { return mom_tiles_of(s); }

hipError_t launch_mom_pivot(int dt, const TaskRef<PartSeg> &tasks, uint32_t tiles,
                            uint32_t overflow, bool init, const Workspace &ws, hipStream_t st) {
    if (tasks.A == 0 || tiles == 0) return hipSuccess;
    switch (dt) {
    case 0: return mom_t<OrdU32>(tasks, tiles, overflow, init, ws, st);
    case 1: return mom_t<OrdF32>(tasks, tiles, overflow, init, ws, st);
    case 2: return mom_t<OrdU64>(tasks, tiles, overflow, init, ws, st);
    case 3: return mom_t<OrdF64>(tasks, tiles, overflow, init, ws, st);
    // the log order is the integers' order: the radix select on the key bits
    case 4: return mom_t<OrdU32>(tasks, tiles, overflow, init, ws, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qms
