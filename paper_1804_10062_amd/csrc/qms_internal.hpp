// qms_internal.hpp -- host-side interfaces between the C ABI / driver and the
// kernel launchers.  Not part of the public interface (include/qms.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qms {

// Fixed capacity of the merge split array: enough for a mergesorted side of
// up to 2^31 elements (the smaller side of any array of < 2^32 keys).
constexpr uint64_t kMaxSplits = (1ull << 31) / 2048 + 2;
// Capacity of the partition chunk-boundary arrays: at most half of a range of
// < 2^32 keys is misplaced, in chunks of kRankChunk (2048).
constexpr uint64_t kMaxChunks = (1ull << 31) / 2048 + 2;

// Library-owned scratch of one (device, stream): counters and round state.
// Its size does not depend on n.
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    void *block = nullptr;       // one device allocation holding the arrays
    uint32_t *cnt_lt = nullptr;  // [kMaxTiles]
    uint32_t *cnt_eq = nullptr;  // [kMaxTiles]
    uint32_t *eqmv = nullptr;    // [kMaxTiles]
    uint32_t *preL = nullptr;    // [kMaxTiles + 1]
    uint32_t *preR = nullptr;    // [kMaxTiles + 1]
    uint32_t *spL = nullptr;     // [kMaxChunks]
    uint32_t *spR = nullptr;     // [kMaxChunks]
    uint32_t *splits = nullptr;  // [kMaxSplits]
    uint64_t *meta = nullptr;    // [M_COUNT]
    uint64_t *h_meta = nullptr;  // pinned host mirror of meta
};

struct PartitionResult {
    uint64_t pivot, c_lt, c_eq, x_a;
};

hipError_t launch_tile_sort(int dt, bool pairs, uint32_t *keys, uint32_t *vals, uint64_t src,
                            uint64_t dst, uint64_t m, bool swap, hipStream_t st);
hipError_t launch_merge_level(int dt, bool pairs, uint32_t *keys, uint32_t *vals, uint64_t src,
                              uint64_t dst, uint64_t m, uint64_t W, uint32_t *splits,
                              hipStream_t st);
hipError_t run_partition(int dt, bool pairs, uint32_t *keys, uint32_t *vals, uint64_t lo,
                         uint64_t hi, const Workspace &ws, PartitionResult *res,
                         hipStream_t st);

}  // namespace qms
