// qms_internal.hpp -- host-side interfaces between the C ABI / driver and the
// kernel launchers.  Not part of the public interface (include/qms.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "qms_device.hpp"

namespace qms {

// ---- fixed workspace capacities (independent of the number of keys) ---------------
// Segments served by one round of launches; larger batches run in groups.
constexpr uint32_t kCapSegs = 32768;
// Partition tiles of one round (the tile grows beyond kPartSub if needed).
constexpr uint64_t kCapTiles = 1ull << 20;
// Chunk boundaries of one round: each segment reserves ceil(s / 4096) + 2.
constexpr uint64_t kCapChunks = (1ull << 21) + 2ull * kCapSegs + 16;
// Per-wave counts of the partition count (#(< p) in each 64 positions, one
// byte each) for rounds of at most this many positions (2^32 keys at the
// default partition tile; 64 MiB); larger rounds locate their chunk
// boundaries by walking whole tiles, several times slower (the first rounds
// of a batch of 2.2 billion keys: 1.1 ms per split launch instead of about
// 0.15 ms).
constexpr uint64_t kCapGroups = 1ull << 26;
// Merge splits of one level: ceil(m / kMergeTile) per task, m < 2^31.
constexpr uint64_t kCapSplits = (1ull << 31) / kMergeTile + kCapSegs + 16;
// Segments whose median-of-medians pivot one launch group selects.
constexpr uint32_t kCapMoM = 2048;
// Merge levels a task can need: ceil(log2(2^31 / 8192)).
constexpr int kMaxLevels = 18;
// Ranges of at least kHugeRange keys are partitioned as blocks of at most
// kHugeBlock keys (qms_huge.hip).  An array may hold up to kMaxSortKeys keys:
// its Mergesort sides (at most half of a range) then stay within the merge
// tables of a workspace (kCapSplits tiles of kMergeTile keys).
#ifndef QMS_HUGE_RANGE_LOG2
#define QMS_HUGE_RANGE_LOG2 32
#endif
#ifndef QMS_HUGE_BLOCK_LOG2
#define QMS_HUGE_BLOCK_LOG2 31
#endif
constexpr uint64_t kHugeRange = 1ull << QMS_HUGE_RANGE_LOG2;
constexpr uint64_t kHugeBlock = 1ull << QMS_HUGE_BLOCK_LOG2;
static_assert(kHugeBlock < kHugeRange && kHugeRange <= (1ull << 32), "block partitions");
constexpr uint64_t kMaxSortKeys = (1ull << 32) + (1ull << 25);
// Largest final_tile: ranges of at most this many keys may leave the loop
// for the in-place bitonic network.
constexpr uint64_t kMaxFinalTile = 1ull << 30;

// Capacities of a workspace.  The cached workspaces take the constants
// above; the allocation-free entry point carves a smaller set for one array
// of bounded size out of a fixed device array.
struct WsCaps {
    uint64_t tiles, chunks, splits, groups;
    uint32_t segs, mom;
    uint32_t rounds;     // segments of a device-controlled batch group (0: none)
    size_t tab_bytes;    // bytes of one task-table arena
};
WsCaps default_caps();
// Caps for one array of at most nmax elements (no batch round state).
WsCaps single_array_caps(uint64_t nmax);
// Device bytes of a workspace with these caps (one block).
size_t workspace_device_bytes(const WsCaps &c);

// Library-owned scratch of one (device, stream): counters, round state and
// task tables.  Its size does not depend on the number of keys sorted.  One
// sort at a time uses it: callers hold `mu` for the whole sort (a
// WorkspaceLease), and `users` counts the leases taken or waiting, so that
// qms_release_workspaces never frees a workspace in use.
struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::atomic<int> users{0};
    void *block = nullptr;       // one device allocation holding everything below
    uint32_t *cnt_lt = nullptr;  // [kCapTiles]
    uint32_t *cnt_eq = nullptr;  // [kCapTiles]
    uint32_t *eqmv = nullptr;    // [kCapTiles]
    uint32_t *preL = nullptr;    // [kCapTiles + kCapSegs]
    uint32_t *preR = nullptr;    // [kCapTiles + kCapSegs]
    uint32_t *spL = nullptr;     // [kCapChunks]
    uint32_t *spR = nullptr;     // [kCapChunks]
    uint32_t *splits = nullptr;  // [kCapSplits]
    // [2 kSamplesPerTile kCapSplits] each: run samples (keys of either
    // width), by pass parity
    uint32_t *samples[2] = {nullptr, nullptr};
    uint32_t *bounds = nullptr;        // [4 * kCapSplits] 4-way pass: tile starts
    uint32_t *ends = nullptr;          // [8 * kCapSplits] 4-way pass: tiles in merge order
    uint64_t *meta = nullptr;    // [kCapSegs * M_COUNT]
    uint32_t *res = nullptr;     // [4 * kCapSegs] per-segment partition results
    uint32_t *hist = nullptr;    // [256 * kCapMoM] median-of-medians select histograms
    uint8_t *gcnt = nullptr;     // [kCapGroups] #(< p) per 64 positions of a partition
    // task tables: device copies of the host arena below
    void *dtab = nullptr;        // [tab_bytes]
    void *htab[2] = {nullptr, nullptr};  // pinned host arenas (alternating rounds)
    // recorded on the stream after the last round that used each host arena:
    // its asynchronous uploads have run once the event has
    hipEvent_t arena_done[2] = {nullptr, nullptr};
    bool arena_busy[2] = {false, false};
    size_t tab_bytes = 0;
    uint32_t *h_res = nullptr;   // pinned host mirror of res
    uint64_t rounds = 0;         // rounds run with this workspace (arena parity)
    WsCaps caps{};
    // device-side round control (qms_rounds.hip): segment states, task
    // tables, prefixes, work counters and the schedule status (errors,
    // unsorted segments), for caps.rounds segments
    void *r_seg = nullptr;
    uint32_t *r_aseg = nullptr;
    uint32_t *r_live[2] = {nullptr, nullptr};  // live lists of alternate rounds
    void *r_ptab = nullptr, *r_mtab = nullptr, *r_stab = nullptr;
    uint32_t *r_pre = nullptr, *r_work = nullptr, *r_status = nullptr;
    // the bitonic network after the last round: work-item prefixes of every
    // pass (kMaxNetPasses arrays) and each pass's item count
    uint32_t *r_netpre = nullptr, *r_netw = nullptr;
    uint32_t *r_blk = nullptr;  // per-workgroup sums of the plans
};
// Device bytes of the round-control state for `segs` segments, and its
// arrays carved out of `b`.
size_t rounds_state_bytes(uint32_t segs);
void carve_rounds_state(Workspace *ws, char *b, uint32_t segs);
// Point every device array of `ws` into `block` (workspace_device_bytes(c)
// bytes, 256-byte aligned) and set its caps.
void carve_workspace(Workspace *ws, char *block, const WsCaps &c);

// Layout of a task-table arena (offsets in bytes; same on host and device).
struct TabLayout {
    size_t part_tab, pre_count, pre_chunk_a, pre_wave_a, pre_chunk_b, pre_wave_b;
    size_t sort_tab, pre_tile, pre_level;  // pre_level: kMaxLevels arrays
    size_t total;
};
TabLayout tab_layout();

// One partition phase launch.
struct PartitionLaunch {
    int phase;                 // 0 count, 6 scanA, 1 splitA, 2 swapA, 3 splitB, 4 scanB, 5 swapB
    TaskRef<PartSeg> tasks;    // table + work prefix of the phase
    uint32_t grid;             // workgroups launched (0: nothing to launch)
    uint32_t first = 0;        // first item (the overflow launch of a device-sized phase)
    bool loop = false;         // the workgroups loop over the items from first on
    uint32_t work;             // waves of a host-sized split launch
    uint32_t TP;               // partition tile
    bool groups;               // count A records per-64-position counts (gcnt)
    uint32_t chunk_span;       // target positions per exchange chunk
    uint32_t scan_threads;     // block size of the scans
    double keys_total;         // keys in all ranges (byte figures)
    double bytes;              // algorithmic bytes of the launch (swap A)
    const Workspace *ws;
};

hipError_t launch_partition_phase(int dt, bool pairs, const PartitionLaunch &L, hipStream_t st);
// Median-of-medians pivots (into meta[M_PIVOT]) of the segments listed in
// `tasks` (PartSeg.pad = histogram slot < kCapMoM); `tiles` = total of
// mom_tiles(s) over them, the exclusive prefix of which is tasks.pre.
uint32_t mom_tiles(uint64_t s);
// (overflow: looping workgroups after each pass of a device-sized launch)
hipError_t launch_mom_pivot(int dt, const TaskRef<PartSeg> &tasks, uint32_t tiles,
                            uint32_t overflow, bool init, const Workspace &ws, hipStream_t st);
hipError_t launch_tile_sort(int dt, bool pairs, const TaskRef<SortSeg> &tasks, uint32_t tiles,
                            uint32_t overflow, double bytes, const Workspace &ws,
                            hipStream_t st);
// One pass of the bitonic network that sorts the loop's last ranges in
// place (qms_bitonic.hip): the mirror step of stage k, the half-cleaner
// steps 2^hi .. 2^lo (j >= T), or the steps below T inside each tile.
// tasks: the ranges (keys, vals, m), tiles already sorted by the base case.
struct BitonicLaunch {
    enum Kind : uint32_t { MIRROR = 0, COLUMNS = 1, TILE = 2, MIRROR_COLUMNS = 3 };
    TaskRef<SortSeg> tasks;
    uint32_t kind = 0, k = 0, lo = 0, hi = 0;
    // workgroups: the sum over the tasks of bitonic_items (host-sized), or
    // with tasks.dyn holding that sum, workgroups that loop over the items
    uint32_t items = 0;
    double bytes = 0;
};
// Threads of the mirror and column kernels, and mirror pairs per workgroup.
constexpr uint32_t kBitThreads = 256;
constexpr uint32_t kMirrorChunk = kBitThreads * 8;
// The passes of the network for ranges of at most 2^K keys whose tiles of
// 2^lt keys are sorted: for every stage k > lt the mirror step with the
// first (up to four) half-cleaner steps 2^(k-2) .. in one pass, the further
// steps down to 2^lt four at a time, the in-tile steps.
std::vector<BitonicLaunch> bitonic_passes(uint32_t K, uint32_t lt);
// Most passes of one network (ranges below 2^33 keys, tiles of at least 2^13).
constexpr uint32_t kMaxNetPasses = 96;
// Workgroups of a range of m keys in a pass (base tile T); 0 for the passes
// of stages above ceil(log2 m), which a range of m keys does not need.
__host__ __device__ inline uint32_t bitonic_items_of(uint32_t kind, uint32_t k, uint32_t lo,
                                                     uint32_t hi, uint64_t m, uint32_t T) {
    if (m <= T || (1ull << (k - 1)) >= m) return 0;
    switch (kind) {
    case BitonicLaunch::MIRROR: {
        // the lower-half positions of every 2^k block the range reaches
        const uint64_t H = 1ull << (k - 1), B = 2 * H;
        const uint64_t pairs = (m + B - 1) / B * H;
        return (uint32_t)((pairs + kMirrorChunk - 1) / kMirrorChunk);
    }
    case BitonicLaunch::COLUMNS: {
        const uint64_t blocks = (m + (1ull << (hi + 1)) - 1) >> (hi + 1);
        return (uint32_t)(blocks * ((1ull << lo) / kBitThreads));
    }
    case BitonicLaunch::MIRROR_COLUMNS: {
        // one thread per column of the lower half of every 2^k block (it
        // also holds the mirrored column of the upper half)
        const uint64_t blocks = (m + (1ull << k) - 1) >> k;
        return (uint32_t)(blocks * ((1ull << lo) / kBitThreads));
    }
    case BitonicLaunch::TILE:
        return (uint32_t)((m + T - 1) / T);
    default:
        return 0;
    }
}
// The in-tile half-cleaners of that network: the base case's last stage on
// each tile (items: the tiles of all tasks).
hipError_t launch_tile_merge(int dt, bool pairs, const TaskRef<SortSeg> &tasks, uint32_t items,
                             hipStream_t st);
hipError_t launch_bitonic_pass(int dt, bool pairs, const BitonicLaunch &L, hipStream_t st);
// Ranges of 2^32 keys or more (qms_huge.hip): the median of three of
// [keys, keys + s) as the pivot of the `blocks` round-state slots from
// slot0 on; the rotation of [a, c) at b (so that [b, c) comes before [a, b)),
// positions in keys of the key width (wide: 64 bits), payloads alike.
hipError_t launch_huge_pivot(int dt, const uint32_t *keys_words, uint64_t s, uint64_t *meta,
                             uint32_t slot0, uint32_t blocks, hipStream_t st);
hipError_t launch_rotate(bool wide, bool pairs, uint32_t *keys_words, uint32_t *vals, uint64_t a,
                         uint64_t b, uint64_t c, hipStream_t st);
// One merge pass (2-way or 4-way) of the tasks listed: every task's pass at
// binary level `level`, or with `step` the step-th pass of every task (its
// level from its level count).  tiles: merge tiles of the listed tasks
// (with tasks.dyn holding the count: the launch's estimate of it).
struct MergeLaunch {
    TaskRef<SortSeg> tasks;
    uint32_t level = 0, step = 0;
    bool four_way = false;
    uint32_t tiles = 0;     // merge tiles (device-sized: the estimate)
    uint32_t overflow = 0;  // device-sized: looping workgroups for tiles beyond it
    double bytes = 0;
};
hipError_t launch_merge_pass(int dt, bool pairs, const MergeLaunch &M, const Workspace &ws,
                             hipStream_t st);

}  // namespace qms
