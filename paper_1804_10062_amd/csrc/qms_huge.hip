// qms_huge.hip -- partition rounds of ranges of 2^32 keys or more.
//
// The partition kernels address a range with 32-bit positions.  A range of
// at least 2^32 keys is partitioned as several blocks of at most 2^31 keys
// around one pivot, the median of three of the whole range (Fig. 2's rule:
// its first, middle and last key); each block comes out as [< p | == p | > p]
// and block rotations then gather the classes: [< p ... | == p ... | > p ...]
// over the whole range.  A rotation of [a, c) at b (so that [b, c) comes
// before [a, b)) reverses [a, b), [b, c) and then [a, c); every reversal
// exchanges cells of the range only, so the round stays in place.  The sides
// it leaves are then sorted by the ordinary Mergesort tasks (at most half the
// range, below 2^32 keys for the array sizes the library accepts).
#include "qms_device.hpp"
#include "qms_internal.hpp"

namespace qms {

namespace {

constexpr int kRevThreads = 256;
constexpr uint32_t kRevPer = 4;  // pairs per thread
constexpr uint64_t kRevChunk = (uint64_t)kRevThreads * kRevPer;

// The pivot of the whole range (order-mapped median of the three sample
// keys) into the M_PIVOT word of each block's round state.
template <class O>
__global__ void k_huge_pivot(const typename O::K *keys, uint64_t s, uint64_t *meta_all,
                             uint32_t slot0, uint32_t blocks) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const auto p = median3_by<O>(O::ord(keys[0]), O::ord(keys[s / 2]), O::ord(keys[s - 1]));
    for (uint32_t b = 0; b < blocks; ++b) meta_all[(uint64_t)(slot0 + b) * M_COUNT + M_PIVOT] = p;
}

// Reverse [0, len) of keys (and payloads): cell i exchanges with len-1-i.
template <class K, bool PAIRS>
__global__ __launch_bounds__(kRevThreads) void k_reverse(K *keys, uint32_t *vals, uint64_t len) {
    const uint64_t half = len / 2;
#pragma unroll
    for (uint32_t q = 0; q < kRevPer; ++q) {
        const uint64_t i = (uint64_t)blockIdx.x * kRevChunk + (uint64_t)q * kRevThreads + threadIdx.x;
        if (i >= half) continue;
        const uint64_t j = len - 1 - i;
        const K x = keys[i], y = keys[j];
        keys[i] = y;
        keys[j] = x;
        if (PAIRS) {
            const uint32_t u = vals[i], v = vals[j];
            vals[i] = v;
            vals[j] = u;
        }
    }
}

template <class K, bool PAIRS>
hipError_t reverse_t(uint32_t *keys_words, uint32_t *vals, uint64_t len, hipStream_t st) {
    if (len < 2) return hipSuccess;
    const uint64_t grid = (len / 2 + kRevChunk - 1) / kRevChunk;
    if (grid > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_reverse<K, PAIRS>), dim3((uint32_t)grid), dim3(kRevThreads), 0, st,
                       (K *)keys_words, vals, len);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_huge_pivot(int dt, const uint32_t *keys_words, uint64_t s, uint64_t *meta,
                             uint32_t slot0, uint32_t blocks, hipStream_t st) {
    switch (dt) {
    case 0:
        hipLaunchKernelGGL(k_huge_pivot<OrdU32>, dim3(1), dim3(64), 0, st, keys_words, s, meta,
                           slot0, blocks);
        break;
    case 4:
        hipLaunchKernelGGL(k_huge_pivot<OrdLogU32>, dim3(1), dim3(64), 0, st, keys_words, s,
                           meta, slot0, blocks);
        break;
    case 1:
        hipLaunchKernelGGL(k_huge_pivot<OrdF32>, dim3(1), dim3(64), 0, st, keys_words, s, meta,
                           slot0, blocks);
        break;
    case 2:
        hipLaunchKernelGGL(k_huge_pivot<OrdU64>, dim3(1), dim3(64), 0, st,
                           (const uint64_t *)keys_words, s, meta, slot0, blocks);
        break;
    case 3:
        hipLaunchKernelGGL(k_huge_pivot<OrdF64>, dim3(1), dim3(64), 0, st,
                           (const uint64_t *)keys_words, s, meta, slot0, blocks);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rotate(bool wide, bool pairs, uint32_t *keys_words, uint32_t *vals, uint64_t a,
                         uint64_t b, uint64_t c, hipStream_t st) {
    if (a >= b || b >= c) return hipSuccess;  // one part empty: nothing moves
    const uint64_t ew = wide ? 2 : 1;
    auto rev = [&](uint64_t x, uint64_t y) -> hipError_t {
        uint32_t *k = keys_words + ew * x;
        uint32_t *v = pairs ? vals + x : nullptr;
        if (wide)
            return pairs ? reverse_t<uint64_t, true>(k, v, y - x, st)
                         : reverse_t<uint64_t, false>(k, v, y - x, st);
        return pairs ? reverse_t<uint32_t, true>(k, v, y - x, st)
                     : reverse_t<uint32_t, false>(k, v, y - x, st);
    };
    hipError_t e = rev(a, b);
    if (e == hipSuccess) e = rev(b, c);
    if (e == hipSuccess) e = rev(a, c);
    return e;
}

}  // namespace qms
