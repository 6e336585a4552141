// qms_host.hpp -- host helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <string>
#include <vector>

#include "qms_internal.hpp"

namespace qms {

// Words per round of the schedule log (QMS_SCHEDULE_WORDS in qms.h).
constexpr int kScheduleWords = 6;

// Run-time tunables (qms_set_tuning): merge arity of key-only sorts, the
// first partition counting tile, the target positions per exchange chunk,
// the Mergesort's base-case run width (QuickMergeXsort's X_THRESH), the
// size at or below which a range leaves the loop for the in-place network.
struct Tuning {
    uint32_t merge_ways = 4;
    uint32_t partition_tile = kPartSub;
    uint32_t chunk_span = (uint32_t)kChunkSpan;
    uint32_t base_tile = 0;   // automatic
    uint32_t final_tile = 0;  // automatic
};
Tuning current_tuning();
// The loop's exit size for keys of type dt: final_tile, or when automatic
// the size measured fastest for that type: 2^24 keys for 32-bit keys (with
// or without payloads), 2^23 for 64-bit keys, whose network passes move
// twice the bytes, and 2^22 for the logarithm comparison, whose network
// comparisons are what the time goes to.  Measured on 2^28 uint32 keys
// (25.3, 25.8, 25.5 Gkeys/s at 2^23, 2^24, 2^25), 2^26 key/payload pairs
// (9.8, 10.0, 10.3, 9.4 at 2^22 .. 2^25), 2^27 uint64 keys (11.02, 11.09,
// 10.90, 10.16 at 2^22 .. 2^25) and 2^26 keys by logarithm (1.34, 1.44,
// 1.56, 1.54, 1.44 at 2^20 .. 2^24).
inline uint64_t loop_exit_keys(const Tuning &t, int dt) {
    if (t.final_tile) return t.final_tile;
    if (dt == 4) return 1ull << 22;
    return (dt == 2 || dt == 3) ? (1ull << 23) : (1ull << 24);
}
// The automatic exit size of one loop over several arrays of lengths
// len[0..count) whose one-array exit size is `one`.  A round's fixed costs
// (its launches and the counters read back) are paid once for all of them,
// and so are the network's.  The group keeps looping while its arrays still
// in the loop hold enough keys together to make a round worth those costs:
// the smallest power of two p >= T0 with (arrays longer than p) * p at
// least four times `one` (the factor measured on batches of serving
// requests: batches of tens of requests keep the one-array size, saturated
// batches of hundreds leave at about 2^18 keys), else `one`.
inline uint64_t group_loop_exit(uint64_t one, uint64_t T0, const uint64_t *len, size_t count) {
    for (uint64_t p = T0; p < one; p *= 2) {
        uint64_t longer = 0;
        for (size_t i = 0; i < count; ++i) longer += len[i] > p;
        if (longer * p >= 4 * one) return p;
    }
    return one;
}

int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *where);
int check_device_ptr(const void *p, const char *what, int *device, uintptr_t align = 4);
// dtype codes of qms.h: 32-bit (QMS_U32, QMS_F32) or 64-bit (QMS_U64, QMS_F64)
inline bool dtype_known(int dt) { return dt >= 0 && dt <= 4; }
// the log-order comparison sorts keys without payloads
inline bool dtype_takes_payloads(int dt) { return dt != QMS_U32_LOG; }
inline bool dtype_wide(int dt) { return dt == 2 || dt == 3; }
// Exclusive use of the workspace of (device, stream) for one sort: taking
// the lease waits for another thread's sort on the same stream to end.
class WorkspaceLease {
  public:
    WorkspaceLease() = default;
    ~WorkspaceLease() { reset(); }
    WorkspaceLease(const WorkspaceLease &) = delete;
    WorkspaceLease &operator=(const WorkspaceLease &) = delete;
    Workspace *get() const { return ws_; }
    Workspace &operator*() const { return *ws_; }
    void reset();

  private:
    friend int get_workspace(int device, hipStream_t stream, WorkspaceLease *out);
    Workspace *ws_ = nullptr;
};
int get_workspace(int device, hipStream_t stream, WorkspaceLease *out);
// Frees the cached workspaces that no thread holds (a workspace in use is
// left alone: QMS_ERR_INVALID names it).
int release_workspaces();
int release_workspace(int device, hipStream_t stream);

// One array to sort: n keys (and payloads) at device addresses.
struct HostSeg {
    uint32_t *keys;
    uint32_t *vals;  // nullptr for keys only
    uint64_t n;
};

// The QuickMergesort loop for every array of the list, all arrays advancing
// through each phase in one launch.  log: record the per-round schedule.
int sort_segments(int dt, bool pairs, const HostSeg *segs, size_t count, Workspace &ws,
                  hipStream_t st, bool log);
// Bytes of one task-table arena for rounds of up to `segs` segments.
size_t tab_arena_bytes(uint32_t segs);
// The batch with device-side round control (qms_rounds.hip): nseg segments
// [h_off[j], h_off[j + 1]) of keys_base (d_offsets: the same offsets on the
// device), each below 2^32 keys.  Enqueues everything on st and returns.
// loop_exit: a range of at most this many keys leaves the loop and is
// sorted by the bitonic network after the last round (at most the base
// tile: the loop runs down to the base case).
int sort_batch_device_rounds(int dt, bool pairs, char *keys_base, uint32_t *vals_base,
                             const uint64_t *d_offsets, const uint64_t *h_off, uint32_t nseg,
                             uint64_t loop_exit, Workspace &ws, hipStream_t st);
const std::vector<std::array<uint64_t, kScheduleWords>> &last_schedule();
// The median-of-medians pivot of one array (order-mapped key into *pivot;
// keys: the array's first word, 32- or 64-bit keys by dt).
int mom_pivot_of(int dt, const uint32_t *keys, uint64_t n, Workspace &ws, hipStream_t st,
                 uint64_t *pivot);

// Makes `dev` current for the lifetime of the object.
class DeviceScope {
  public:
    explicit DeviceScope(int dev);
    ~DeviceScope();
    DeviceScope(const DeviceScope &) = delete;
    DeviceScope &operator=(const DeviceScope &) = delete;

  private:
    int prev_ = 0, dev_ = 0;
};

}  // namespace qms
