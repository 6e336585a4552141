// qms_noalloc.hip -- qms_sort_noalloc: the single-array sort of qms_sort for
// callers that cannot allocate (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The counters, prefixes, split vectors and run samples that the kernels use
// live in `scratch`, a fixed device array of this file, instead of a cached
// workspace; the host side keeps its small task-table arenas and readback
// words in static host memory.  Nothing is allocated per call: no hipMalloc,
// no hipFree, no pinned host memory, no events.  The array is sized for one
// array of at most kNoAllocMaxKeys keys; the loop's last ranges are sorted
// in place by the bitonic X, as in qms_sort, so no buffer beyond it is
// needed.
//
// Each device holds its own copy of `scratch` at its own address; host code
// takes that address from hipGetSymbolAddress once per device (with the
// device current) and passes it to the kernels like any workspace pointer.
// The array's name itself is a host-side stand-in and is never used as an
// address.  Calls share the array of their device: they are serialised on
// the host, and calls whose GPU work overlaps (different streams of one
// device, not synchronised between the calls) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "qms.h"
#include "qms_host.hpp"
#include "qms_internal.hpp"

namespace qms {
constexpr uint64_t kNoAllocMaxKeys = 1ull << 28;
constexpr size_t kNoAllocScratchBytes = 32ull << 20;  // 32 MiB per device
constexpr int kNoAllocMaxDevices = 64;
}  // namespace qms

static __device__ __align__(256) uint8_t scratch[qms::kNoAllocScratchBytes];

namespace qms {
namespace {

std::mutex g_noalloc_mu;  // host state below, and calls on any device
void *g_scratch_ptr[kNoAllocMaxDevices];
Workspace g_noalloc_ws[kNoAllocMaxDevices];
bool g_noalloc_ready[kNoAllocMaxDevices];
// two task-table arenas and the readback words (pageable, static)
alignas(256) char g_host_arena[2][80 * 1024];
uint32_t g_host_res[4];

// First call on `dev` (current): the device's address of `scratch`, and the
// workspace carved out of it.
int noalloc_setup(int dev) {
    if (g_noalloc_ready[dev]) return QMS_OK;
    const WsCaps caps = single_array_caps(kNoAllocMaxKeys);
    if (workspace_device_bytes(caps) > kNoAllocScratchBytes || caps.tab_bytes > sizeof(g_host_arena[0]))
        return set_error(QMS_ERR_UNSUPPORTED, "allocation-free scratch too small for its key limit");
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return hip_error(e == hipSuccess ? hipErrorInvalidSymbol : e,
                         "hipGetSymbolAddress of the allocation-free scratch");
    }
    g_scratch_ptr[dev] = ptr;
    Workspace &ws = g_noalloc_ws[dev];
    ws.device = dev;
    ws.block = nullptr;  // not owned
    ws.htab[0] = g_host_arena[0];
    ws.htab[1] = g_host_arena[1];
    ws.h_res = g_host_res;
    ws.arena_done[0] = ws.arena_done[1] = nullptr;
    carve_workspace(&ws, (char *)ptr, caps);
    g_noalloc_ready[dev] = true;
    return QMS_OK;
}

}  // namespace
}  // namespace qms

using namespace qms;

extern "C" int qms_sort_noalloc(void *d_keys, uint64_t n, int dt, hipStream_t stream) {
    try {
        if (!dtype_known(dt)) return set_error(QMS_ERR_UNSUPPORTED, "unknown dtype");
        if (n <= 1) return QMS_OK;
        if (d_keys == nullptr) return set_error(QMS_ERR_INVALID, "NULL pointer with n > 1");
        if (n > kNoAllocMaxKeys)
            return set_error(QMS_ERR_UNSUPPORTED,
                             "qms_sort_noalloc takes at most 2^28 keys (its fixed scratch); "
                             "use qms_sort");
        int dev = 0;
        int rc = check_device_ptr(d_keys, "keys", &dev, dtype_wide(dt) ? 8 : 4);
        if (rc != QMS_OK) return rc;
        if (dev < 0 || dev >= kNoAllocMaxDevices)
            return set_error(QMS_ERR_UNSUPPORTED, "device ordinal beyond the allocation-free table");
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        DeviceScope scope(dev);
        rc = noalloc_setup(dev);
        if (rc != QMS_OK) return rc;
        Workspace &ws = g_noalloc_ws[dev];
        ws.stream = stream;
        HostSeg seg{(uint32_t *)d_keys, nullptr, n};
        return sort_segments(dt, false, &seg, 1, ws, stream, true);
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_sort_noalloc");
    }
}
