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

// ---- workspaces ----------------------------------------------------------------------
static std::mutex g_ws_mutex;
static std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

static size_t ws_words() {
    return 3ull * kMaxTiles + 2ull * (kMaxTiles + 1) + 2ull * kMaxChunks + kMaxSplits;
}

int get_workspace(int device, hipStream_t stream, Workspace **out) {
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    auto key = std::make_pair(device, stream);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return QMS_OK;
    }
    Workspace *ws = new Workspace();
    ws->device = device;
    ws->stream = stream;
    const size_t words = ws_words();
    const size_t bytes = words * sizeof(uint32_t) + M_COUNT * sizeof(uint64_t) + 256;
    hipError_t e = hipMalloc(&ws->block, bytes);
    if (e != hipSuccess) {
        delete ws;
        (void)hipGetLastError();
        return set_error(QMS_ERR_NOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
    }
    e = hipHostMalloc((void **)&ws->h_meta, M_COUNT * sizeof(uint64_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(ws->block);
        delete ws;
        (void)hipGetLastError();
        return set_error(QMS_ERR_NOMEM, std::string("pinned host allocation: ") + hipGetErrorString(e));
    }
    uint64_t *meta = (uint64_t *)ws->block;
    uint32_t *w = (uint32_t *)(meta + M_COUNT);
    ws->meta = meta;
    ws->cnt_lt = w;
    w += kMaxTiles;
    ws->cnt_eq = w;
    w += kMaxTiles;
    ws->eqmv = w;
    w += kMaxTiles;
    ws->preL = w;
    w += kMaxTiles + 1;
    ws->preR = w;
    w += kMaxTiles + 1;
    ws->spL = w;
    w += kMaxChunks;
    ws->spR = w;
    w += kMaxChunks;
    ws->splits = w;
    g_ws[key] = ws;
    *out = ws;
    return QMS_OK;
}

int release_workspaces() {
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        Workspace *ws = kv.second;
        (void)hipSetDevice(ws->device);
        (void)hipStreamSynchronize(ws->stream);
        (void)hipFree(ws->block);
        (void)hipHostFree(ws->h_meta);
        delete ws;
    }
    g_ws.clear();
    (void)hipSetDevice(cur);
    return QMS_OK;
}

// ---- argument checks ---------------------------------------------------------------
int check_device_ptr(const void *p, const char *what, int *device) {
    if (((uintptr_t)p & 3u) != 0)
        return set_error(QMS_ERR_ALIGN, std::string(what) + " is not 4-byte aligned");
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

// ---- the QuickMergesort loop ------------------------------------------------------------
static thread_local std::vector<std::array<uint64_t, 5>> g_schedule;

// Mergesort of the m elements at D with the m cells at Bf as swap space
// (Fig. 2's out()/msort()/merge(), bottom-up with power-of-two run widths).
// The base case writes into the buffer when the number of merge levels is
// odd, so that the last level lands in D.  Returns the number of levels.
int mergesort_side(int dt, bool pairs, uint32_t *keys, uint32_t *vals, uint64_t D,
                   uint64_t Bf, uint64_t m, const Workspace &ws, hipStream_t st, int *levels) {
    *levels = 0;
    if (m == 0) return QMS_OK;
    const uint64_t ntiles = (m + kBaseTile - 1) / kBaseTile;
    int L = 0;
    while ((1ull << L) < ntiles) ++L;
    const bool odd = (L & 1) != 0;
    hipError_t e = launch_tile_sort(dt, pairs, keys, vals, D, odd ? Bf : D, m, odd, st);
    if (e != hipSuccess) return hip_error(e, "base case launch");
    uint64_t cur = odd ? Bf : D, oth = odd ? D : Bf;
    uint64_t W = kBaseTile;
    for (int l = 0; l < L; ++l) {
        e = launch_merge_level(dt, pairs, keys, vals, cur, oth, m, W, ws.splits, st);
        if (e != hipSuccess) return hip_error(e, "merge launch");
        std::swap(cur, oth);
        W *= 2;
    }
    *levels = L;
    return QMS_OK;
}

int sort_array(int dt, bool pairs, uint32_t *keys, uint32_t *vals, uint64_t n,
               const Workspace &ws, hipStream_t st, bool log) {
    if (log) g_schedule.clear();
    uint64_t lo = 0, hi = n;
    while (hi - lo > (uint64_t)kBaseTile) {
        PartitionResult pr;
        hipError_t e = run_partition(dt, pairs, keys, vals, lo, hi, ws, &pr, st);
        if (e != hipSuccess) return hip_error(e, "partition");
        const uint64_t s = hi - lo;
        if (pr.c_lt + pr.c_eq > s || pr.c_eq == 0)
            return set_error(QMS_ERR_HIP, "partition returned inconsistent counts");
        const uint64_t b1 = lo + pr.c_lt, b2 = b1 + pr.c_eq;
        const uint64_t mL = pr.c_lt, mR = hi - b2;
        int levels = 0, rc;
        if (mL <= mR) {
            rc = mergesort_side(dt, pairs, keys, vals, lo, b2, mL, ws, st, &levels);
            lo = b2;
        } else {
            rc = mergesort_side(dt, pairs, keys, vals, b2, b1 - mR, mR, ws, st, &levels);
            hi = b1;
        }
        if (rc != QMS_OK) return rc;
        if (log) g_schedule.push_back({s, pr.c_lt, pr.c_eq, s - pr.c_lt - pr.c_eq, (uint64_t)levels});
    }
    if (hi - lo > 1) {
        hipError_t e = launch_tile_sort(dt, pairs, keys, vals, lo, lo, hi - lo, false, st);
        if (e != hipSuccess) return hip_error(e, "final base case launch");
    }
    return QMS_OK;
}

static int sort_entry(void *d_keys, uint32_t *d_vals, uint64_t n, int dt, hipStream_t stream,
                      bool pairs) {
    if (dt != QMS_U32 && dt != QMS_F32) return set_error(QMS_ERR_UNSUPPORTED, "unknown dtype");
    if (n <= 1) return QMS_OK;
    if (d_keys == nullptr || (pairs && d_vals == nullptr))
        return set_error(QMS_ERR_INVALID, "NULL pointer with n > 1");
    if (n >= (1ull << 32))
        return set_error(QMS_ERR_UNSUPPORTED, "n must be below 2^32");
    int dev = 0, dev2 = 0;
    int rc = check_device_ptr(d_keys, "keys", &dev);
    if (rc != QMS_OK) return rc;
    if (pairs) {
        rc = check_device_ptr(d_vals, "vals", &dev2);
        if (rc != QMS_OK) return rc;
        if (dev2 != dev) return set_error(QMS_ERR_INVALID, "keys and vals on different devices");
    }
    DeviceScope scope(dev);
    Workspace *ws = nullptr;
    rc = get_workspace(dev, stream, &ws);
    if (rc != QMS_OK) return rc;
    return sort_array(dt, pairs, (uint32_t *)d_keys, d_vals, n, *ws, stream, true);
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

uint64_t qms_last_schedule(uint64_t *out, uint64_t max_rounds) {
    const uint64_t n = g_schedule.size();
    if (out) {
        for (uint64_t i = 0; i < n && i < max_rounds; ++i)
            for (int j = 0; j < 5; ++j) out[i * 5 + j] = g_schedule[i][j];
    }
    return n;
}

void qms_get_tiles(uint32_t *base_tile, uint32_t *merge_tile, uint32_t *partition_tile) {
    if (base_tile) *base_tile = kBaseTile;
    if (merge_tile) *merge_tile = kMergeTile;
    if (partition_tile) *partition_tile = kPartSub;
}

}  // extern "C"
