// qms_api.cpp -- the C ABI of libqms.so and the host driver of the
// QuickMergesort loop (Fig. 2's sort(): partition, Mergesort the smaller side
// with the larger side as swap space, continue on the larger side).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "qms.h"
#include "qms_device.hpp"
#include "qms_internal.hpp"
#include "qms_host.hpp"

namespace qms {

// ---- errors ------------------------------------------------------------------------
static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int hip_error(hipError_t e, const char *where) {
    return set_error(QMS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// ---- run-time tuning -------------------------------------------------------------------
static std::mutex g_tuning_mutex;
static Tuning g_tuning;

Tuning current_tuning() {
    std::lock_guard<std::mutex> lock(g_tuning_mutex);
    return g_tuning;
}

// ---- workspaces ----------------------------------------------------------------------
static std::mutex g_ws_mutex;
static std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

WsCaps default_caps() {
    WsCaps c;
    c.tiles = kCapTiles;
    c.chunks = kCapChunks;
    c.splits = kCapSplits;
    c.groups = kCapGroups;
    c.segs = kCapSegs;
    // one histogram per segment: a device-controlled round may give every
    // segment of a group the median-of-medians pivot
    c.mom = kCapSegs;
    c.rounds = kCapSegs;
    c.tab_bytes = tab_arena_bytes(kCapSegs);
    return c;
}

WsCaps single_array_caps(uint64_t nmax) {
    WsCaps c;
    c.tiles = (nmax + kPartSub - 1) / kPartSub + 1;
    c.chunks = c.tiles + 2 + 16;
    c.splits = (nmax + kMergeTile - 1) / kMergeTile + 1 + 16;
    c.groups = c.tiles * (kPartSub / kWave);
    c.segs = 1;
    c.mom = 1;
    c.rounds = 0;
    c.tab_bytes = tab_arena_bytes(1);
    return c;
}

static size_t ws_words(const WsCaps &c) {
    return 3ull * c.tiles + 2ull * (c.tiles + c.segs) + 2ull * c.chunks +
           (13ull + 4ull * kSamplesPerTile) * c.splits + 4ull * c.segs + 256ull * c.mom +
           (c.groups + 3) / 4;
}

size_t workspace_device_bytes(const WsCaps &c) {
    const size_t meta_bytes = (size_t)c.segs * M_COUNT * sizeof(uint64_t);
    const size_t rounds_bytes = c.rounds ? rounds_state_bytes(c.rounds) : 0;
    return meta_bytes + ((c.tab_bytes + 255) & ~(size_t)255) + rounds_bytes +
           ws_words(c) * sizeof(uint32_t) + 256;
}

void carve_workspace(Workspace *ws, char *block, const WsCaps &c) {
    ws->caps = c;
    ws->tab_bytes = c.tab_bytes;
    char *b = block;
    ws->meta = (uint64_t *)b;
    b += (size_t)c.segs * M_COUNT * sizeof(uint64_t);
    ws->dtab = b;
    b += (c.tab_bytes + 255) & ~(size_t)255;
    if (c.rounds) {
        carve_rounds_state(ws, b, c.rounds);
        b += rounds_state_bytes(c.rounds);
    }
    uint32_t *w = (uint32_t *)b;
    ws->cnt_lt = w;
    w += c.tiles;
    ws->cnt_eq = w;
    w += c.tiles;
    ws->eqmv = w;
    w += c.tiles;
    ws->preL = w;
    w += c.tiles + c.segs;
    ws->preR = w;
    w += c.tiles + c.segs;
    ws->spL = w;
    w += c.chunks;
    ws->spR = w;
    w += c.chunks;
    ws->splits = w;
    w += c.splits;
    // run samples hold keys of either width: 2 words per entry (8-byte
    // aligned: every offset before them is a multiple of 8 bytes)
    if ((uintptr_t)w & 7) ++w;
    ws->samples[0] = w;
    w += 2ull * kSamplesPerTile * c.splits;
    ws->samples[1] = w;
    w += 2ull * kSamplesPerTile * c.splits;
    ws->bounds = w;
    w += 4ull * c.splits;
    ws->ends = w;
    w += 8ull * c.splits;
    ws->res = w;
    w += 4ull * c.segs;
    ws->hist = w;
    w += 256ull * c.mom;
    ws->gcnt = (uint8_t *)w;
}

void WorkspaceLease::reset() {
    if (ws_) {
        ws_->mu.unlock();
        ws_->users.fetch_sub(1);
        ws_ = nullptr;
    }
}

static int create_workspace(int device, hipStream_t stream, Workspace **out);

int get_workspace(int device, hipStream_t stream, WorkspaceLease *lease) {
    lease->reset();
    Workspace *ws = nullptr;
    {
        // the user count is raised under the map's lock, so that a release
        // (which holds that lock) sees every lease taken or waiting
        std::lock_guard<std::mutex> lock(g_ws_mutex);
        auto key = std::make_pair(device, stream);
        auto it = g_ws.find(key);
        if (it != g_ws.end()) {
            ws = it->second;
        } else {
            int rc = create_workspace(device, stream, &ws);
            if (rc != QMS_OK) return rc;
            g_ws[key] = ws;
        }
        ws->users.fetch_add(1);
    }
    ws->mu.lock();  // waits for another thread's sort on this stream
    lease->ws_ = ws;
    return QMS_OK;
}

static int create_workspace(int device, hipStream_t stream, Workspace **out) {
    Workspace *ws = new Workspace();
    ws->device = device;
    ws->stream = stream;
    const WsCaps caps = default_caps();
    hipError_t e = hipMalloc(&ws->block, workspace_device_bytes(caps));
    if (e != hipSuccess) {
        delete ws;
        (void)hipGetLastError();
        return set_error(QMS_ERR_NOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
    }
    void *h = nullptr;
    e = hipHostMalloc(&h, 2 * caps.tab_bytes + 4 * (size_t)caps.segs * sizeof(uint32_t),
                      hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(ws->block);
        delete ws;
        (void)hipGetLastError();
        return set_error(QMS_ERR_NOMEM, std::string("pinned host allocation: ") + hipGetErrorString(e));
    }
    for (hipEvent_t &ev : ws->arena_done) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (hipEvent_t &x : ws->arena_done)
                if (x) (void)hipEventDestroy(x);
            (void)hipHostFree(h);
            (void)hipFree(ws->block);
            delete ws;
            (void)hipGetLastError();
            return set_error(QMS_ERR_NOMEM, std::string("event creation: ") + hipGetErrorString(e));
        }
    }
    ws->htab[0] = h;
    ws->htab[1] = (char *)h + caps.tab_bytes;
    ws->h_res = (uint32_t *)((char *)h + 2 * caps.tab_bytes);
    carve_workspace(ws, (char *)ws->block, caps);
    // the median-of-medians histograms and the round status start at zero
    // (device-controlled rounds rely on each select leaving its histogram
    // cleared)
    e = hipMemsetAsync(ws->hist, 0, 256ull * caps.mom * sizeof(uint32_t), stream);
    if (e == hipSuccess && ws->r_status)
        e = hipMemsetAsync(ws->r_status, 0, 4 * sizeof(uint32_t), stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        for (hipEvent_t &x : ws->arena_done) (void)hipEventDestroy(x);
        (void)hipHostFree(h);
        (void)hipFree(ws->block);
        delete ws;
        return hip_error(e, "workspace initialisation");
    }
    *out = ws;
    return QMS_OK;
}

static void free_workspace(Workspace *ws) {
    (void)hipSetDevice(ws->device);
    (void)hipStreamSynchronize(ws->stream);
    for (hipEvent_t &e : ws->arena_done)
        if (e) (void)hipEventDestroy(e);
    (void)hipFree(ws->block);
    (void)hipHostFree(ws->htab[0]);
    delete ws;
}

// Callers hold g_ws_mutex, so no lease can be taken meanwhile; a workspace
// with users is in use (or about to be) and stays.
int release_workspace(int device, hipStream_t stream) {
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    auto it = g_ws.find(std::make_pair(device, stream));
    if (it == g_ws.end()) return QMS_OK;
    if (it->second->users.load() != 0)
        return set_error(QMS_ERR_INVALID, "the workspace of this stream is in use");
    int cur = 0;
    (void)hipGetDevice(&cur);
    free_workspace(it->second);
    g_ws.erase(it);
    (void)hipSetDevice(cur);
    return QMS_OK;
}

int release_workspaces() {
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    bool busy = false;
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (it->second->users.load() != 0) {
            busy = true;
            ++it;
            continue;
        }
        free_workspace(it->second);
        it = g_ws.erase(it);
    }
    (void)hipSetDevice(cur);
    if (busy) return set_error(QMS_ERR_INVALID, "a workspace in use (a running sort or server) was kept");
    return QMS_OK;
}

// ---- argument checks ---------------------------------------------------------------
int check_device_ptr(const void *p, const char *what, int *device, uintptr_t align) {
    if (((uintptr_t)p & (align - 1)) != 0)
        return set_error(QMS_ERR_ALIGN, std::string(what) + " is not " + std::to_string(align) +
                                            "-byte aligned");
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof(a));
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(QMS_ERR_INVALID, std::string(what) + " is not HIP device memory");
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return set_error(QMS_ERR_INVALID, std::string(what) + " is not device memory");
    *device = a.device;
    return QMS_OK;
}

DeviceScope::DeviceScope(int dev) {
    (void)hipGetDevice(&prev_);
    if (prev_ != dev) (void)hipSetDevice(dev);
    dev_ = dev;
}
DeviceScope::~DeviceScope() {
    if (prev_ != dev_) (void)hipSetDevice(prev_);
}

static int sort_entry(void *d_keys, uint32_t *d_vals, uint64_t n, int dt, hipStream_t stream,
                      bool pairs) {
    if (!dtype_known(dt)) return set_error(QMS_ERR_UNSUPPORTED, "unknown dtype");
    if (pairs && !dtype_takes_payloads(dt))
        return set_error(QMS_ERR_UNSUPPORTED, "QMS_U32_LOG sorts keys without payloads");
    if (n <= 1) return QMS_OK;
    if (d_keys == nullptr || (pairs && d_vals == nullptr))
        return set_error(QMS_ERR_INVALID, "NULL pointer with n > 1");
    if (n > kMaxSortKeys)
        return set_error(QMS_ERR_UNSUPPORTED, "n must be at most 2^32 + 2^25");
    int dev = 0, dev2 = 0;
    int rc = check_device_ptr(d_keys, "keys", &dev, dtype_wide(dt) ? 8 : 4);
    if (rc != QMS_OK) return rc;
    if (pairs) {
        rc = check_device_ptr(d_vals, "vals", &dev2);
        if (rc != QMS_OK) return rc;
        if (dev2 != dev) return set_error(QMS_ERR_INVALID, "keys and vals on different devices");
    }
    DeviceScope scope(dev);
    WorkspaceLease ws;
    rc = get_workspace(dev, stream, &ws);
    if (rc != QMS_OK) return rc;
    // Under stream capture nothing may be read back: the rounds are planned
    // on the device, as for a batch of one array, whose last range (at most
    // final_tile keys) the bitonic network sorts, as the host-planned loop
    // does.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (stream != nullptr && hipStreamIsCapturing(stream, &cap) == hipSuccess &&
        cap == hipStreamCaptureStatusActive) {
        if (n >= kHugeRange)
            return set_error(QMS_ERR_UNSUPPORTED, "a captured sort takes fewer than 2^32 keys");
        const uint64_t h_off[2] = {0, n};
        return sort_batch_device_rounds(dt, pairs, (char *)d_keys, pairs ? d_vals : nullptr,
                                        nullptr, h_off, 1, loop_exit_keys(current_tuning(), dt), *ws,
                                        stream);
    }
    HostSeg seg{(uint32_t *)d_keys, pairs ? d_vals : nullptr, n};
    return sort_segments(dt, pairs, &seg, 1, *ws, stream, true);
}

}  // namespace qms

using namespace qms;

extern "C" {

int qms_sort(void *d_keys, uint64_t n, int dt, hipStream_t stream) {
    try {
        return sort_entry(d_keys, nullptr, n, dt, stream, false);
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_sort");
    }
}

int qms_sort_pairs(void *d_keys, uint32_t *d_vals, uint64_t n, int dt, hipStream_t stream) {
    try {
        return sort_entry(d_keys, d_vals, n, dt, stream, true);
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_sort_pairs");
    }
}

const char *qms_last_error(void) { return g_last_error.c_str(); }

int qms_release_workspaces(void) {
    try {
        return release_workspaces();
    } catch (...) {
        return set_error(QMS_ERR_HIP, "host exception in qms_release_workspaces");
    }
}

static_assert(kScheduleWords == QMS_SCHEDULE_WORDS, "schedule record size");

int qms_set_tuning(const qms_tuning *t) {
    if (!t) return set_error(QMS_ERR_INVALID, "NULL tuning");
    if (t->merge_ways != 2 && t->merge_ways != 4)
        return set_error(QMS_ERR_INVALID, "merge_ways must be 2 or 4");
    const uint32_t pt = t->partition_tile;
    if (pt < (uint32_t)kPartSub || pt > 16u * kPartSub || (pt & (pt - 1)) != 0)
        return set_error(QMS_ERR_INVALID, "partition_tile must be a power of two in [4096, 65536]");
    if (t->chunk_span < (uint32_t)kPartSub || t->chunk_span > (1u << 20))
        return set_error(QMS_ERR_INVALID, "chunk_span must lie in [4096, 2^20]");
    const uint32_t bt = t->base_tile;
    if (bt != 0 && (bt < (uint32_t)kMergeTile || bt > kBaseTileKeys || (bt & (bt - 1)) != 0))
        return set_error(QMS_ERR_INVALID, "base_tile must be 0 or a power of two in [2048, 16384]");
    const uint32_t ft = t->final_tile;
    if (ft != 0 && (ft < kBaseTilePairs || ft > kMaxFinalTile || (ft & (ft - 1)) != 0))
        return set_error(QMS_ERR_INVALID, "final_tile must be 0 or a power of two in [8192, 2^30]");
    std::lock_guard<std::mutex> lock(g_tuning_mutex);
    g_tuning.final_tile = ft;
    g_tuning.merge_ways = t->merge_ways;
    g_tuning.partition_tile = pt;
    g_tuning.chunk_span = t->chunk_span;
    g_tuning.base_tile = bt;
    return QMS_OK;
}

int qms_get_tuning(qms_tuning *t) {
    if (!t) return set_error(QMS_ERR_INVALID, "NULL tuning");
    const Tuning c = current_tuning();
    t->merge_ways = c.merge_ways;
    t->partition_tile = c.partition_tile;
    t->chunk_span = c.chunk_span;
    t->base_tile = c.base_tile;
    t->final_tile = c.final_tile;
    return QMS_OK;
}

uint64_t qms_last_schedule(uint64_t *out, uint64_t max_rounds) {
    const auto &sched = last_schedule();
    const uint64_t n = sched.size();
    if (out) {
        for (uint64_t i = 0; i < n && i < max_rounds; ++i)
            for (int j = 0; j < kScheduleWords; ++j) out[i * kScheduleWords + j] = sched[i][j];
    }
    return n;
}

int qms_mom_pivot(const void *d_keys, uint64_t n, int dt, void *pivot_out,
                  hipStream_t stream) {
    try {
        if (!d_keys || !pivot_out) return set_error(QMS_ERR_INVALID, "NULL keys or output");
        if (!dtype_known(dt)) return set_error(QMS_ERR_UNSUPPORTED, "unknown dtype");
        if (n < 3) return set_error(QMS_ERR_INVALID, "the pivot needs n >= 3");
        if (n >= (1ull << 32)) return set_error(QMS_ERR_UNSUPPORTED, "n must be below 2^32");
        const bool wide = dtype_wide(dt);
        int dev = -1;
        int rc = check_device_ptr(d_keys, "keys", &dev, wide ? 8 : 4);
        if (rc != QMS_OK) return rc;
        DeviceScope scope(dev);
        WorkspaceLease ws;
        rc = get_workspace(dev, stream, &ws);
        if (rc != QMS_OK) return rc;
        uint64_t p = 0;
        rc = mom_pivot_of(dt, (const uint32_t *)d_keys, n, *ws, stream, &p);
        if (rc != QMS_OK) return rc;
        // order-mapped key back to the caller's bits (the total order's map
        // undone for floats; integers and the logarithm order map to themselves)
        if (dt == QMS_F32) {
            const uint32_t k = (uint32_t)p;
            p = k ^ ((uint32_t)((int32_t)(~k) >> 31) | 0x80000000u);
        } else if (dt == QMS_F64) {
            p ^= (uint64_t)((int64_t)(~p) >> 63) | 0x8000000000000000ull;
        }
        if (wide) {
            std::memcpy(pivot_out, &p, sizeof(uint64_t));
        } else {
            const uint32_t p32 = (uint32_t)p;
            std::memcpy(pivot_out, &p32, sizeof(uint32_t));
        }
        return QMS_OK;
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_mom_pivot");
    }
}

void qms_get_tiles(uint32_t *base_tile, uint32_t *merge_tile, uint32_t *partition_tile) {
    if (base_tile) *base_tile = kBaseTileKeys;
    if (merge_tile) *merge_tile = kMergeTile;
    if (partition_tile) *partition_tile = kPartSub;
}

}  // extern "C"
