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
#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_prof.hpp"

namespace qms {

// Triples per histogram workgroup (kBlock threads x kMomPerThread).
constexpr int kMomPerThread = 32;
constexpr uint32_t kMomTile = (uint32_t)kBlock * kMomPerThread;

__device__ __forceinline__ const PartSeg &mom_seg(const TaskRef<PartSeg> &r, uint32_t a) {
    return r.A == 1 ? r.one : r.tab[a];
}

// One workgroup per segment: clear the histogram, set rank and prefix.
__global__ __launch_bounds__(kBlock) void k_mom_init(TaskRef<PartSeg> tasks, uint64_t *meta_all,
                                                     uint32_t *hist_all) {
    const PartSeg g = mom_seg(tasks, blockIdx.x);
    stg(hist_all + (uint64_t)g.pad * 256 + threadIdx.x, 0u);
    if (threadIdx.x == 0) {
        uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
        const uint64_t c = g.s / 3;
        meta[M_MOM_RANK] = (c - 1) / 2;
        meta[M_MOM_PREFIX] = 0;
    }
}

// Histogram of digit `pass` (the pass-th byte from the top) of the medians
// whose higher digits equal the prefix chosen so far.
template <class O>
__global__ __launch_bounds__(kBlock) void k_mom_hist(TaskRef<PartSeg> tasks, uint32_t pass,
                                                     const uint64_t *meta_all,
                                                     uint32_t *hist_all) {
    using K = typename O::K;
    constexpr uint32_t kBits = 8 * sizeof(K);
    __shared__ uint32_t h[256];
    uint32_t t, a;
    const PartSeg g = task_of(tasks, blockIdx.x, &t, &a);
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
    if (v != 0) atomicAdd(hist_all + (uint64_t)g.pad * 256 + threadIdx.x, v);
}

// One workgroup per segment: the bucket that holds rank r; the prefix grows
// by its digit and r becomes the rank inside it.  The histogram is cleared
// for the next pass.  After the last pass the prefix is the pivot.
__global__ __launch_bounds__(kBlock) void k_mom_pick(TaskRef<PartSeg> tasks, uint32_t pass,
                                                     uint32_t last, uint64_t *meta_all,
                                                     uint32_t *hist_all) {
    __shared__ uint32_t tmp[kWaves + 1];
    const PartSeg g = mom_seg(tasks, blockIdx.x);
    uint64_t *meta = meta_all + (uint64_t)g.slot * M_COUNT;
    uint32_t *hist = hist_all + (uint64_t)g.pad * 256;
    const uint32_t b = threadIdx.x;
    const uint32_t v = hist[b];
    const uint32_t r = (uint32_t)meta[M_MOM_RANK];
    const uint64_t prefix = meta[M_MOM_PREFIX];
    uint32_t total;
    const uint32_t below = block_exclusive_scan(v, tmp, &total);
    stg(hist + b, 0u);
    if (below <= r && r < below + v) {
        const uint64_t np = (prefix << 8) | b;
        meta[M_MOM_RANK] = r - below;
        meta[M_MOM_PREFIX] = np;
        if (pass == last) meta[M_PIVOT] = np;
    }
}

template <class O>
static hipError_t mom_t(const TaskRef<PartSeg> &tasks, uint32_t tiles, const Workspace &ws,
                        hipStream_t st) {
    ProfScope prof(st, K_PART_SCAN, 0.0);
    constexpr uint32_t kPasses = sizeof(typename O::K);  // 8-bit digits
    hipLaunchKernelGGL(k_mom_init, dim3(tasks.A), dim3(kBlock), 0, st, tasks, ws.meta, ws.hist);
    for (uint32_t pass = 0; pass < kPasses; ++pass) {
        hipLaunchKernelGGL((k_mom_hist<O>), dim3(tiles), dim3(kBlock), 0, st, tasks, pass,
                           (const uint64_t *)ws.meta, ws.hist);
        hipLaunchKernelGGL(k_mom_pick, dim3(tasks.A), dim3(kBlock), 0, st, tasks, pass,
                           kPasses - 1, ws.meta, ws.hist);
    }
    return hipGetLastError();
}

uint32_t mom_tiles(uint64_t s) { return (uint32_t)((s / 3 + kMomTile - 1) / kMomTile); }

hipError_t launch_mom_pivot(int dt, const TaskRef<PartSeg> &tasks, uint32_t tiles,
                            const Workspace &ws, hipStream_t st) {
    if (tasks.A == 0 || tiles == 0) return hipSuccess;
    switch (dt) {
    case 0: return mom_t<OrdU32>(tasks, tiles, ws, st);
    case 1: return mom_t<OrdF32>(tasks, tiles, ws, st);
    case 2: return mom_t<OrdU64>(tasks, tiles, ws, st);
    case 3: return mom_t<OrdF64>(tasks, tiles, ws, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qms
