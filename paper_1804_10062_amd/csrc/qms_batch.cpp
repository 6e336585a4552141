// qms_batch.cpp -- qms_sort_batch: many independent arrays in one call; all
// arrays advance together through the phases of the QuickMergesort loop.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qms.h"
#include "qms_host.hpp"

using namespace qms;

extern "C" int qms_sort_batch(void *d_keys, uint32_t *d_vals, const uint64_t *d_offsets,
                              const uint64_t *h_offsets, uint32_t num_segments, int dt,
                              hipStream_t stream) {
    try {
        if (!dtype_known(dt)) return set_error(QMS_ERR_UNSUPPORTED, "unknown dtype");
        if (d_vals && !dtype_takes_payloads(dt))
            return set_error(QMS_ERR_UNSUPPORTED, "QMS_U32_LOG sorts keys without payloads");
        if (num_segments == 0) return QMS_OK;
        if (d_keys == nullptr || d_offsets == nullptr)
            return set_error(QMS_ERR_INVALID, "NULL keys or offsets");
        int dev = 0, dev2 = 0;
        int rc = check_device_ptr(d_keys, "keys", &dev, dtype_wide(dt) ? 8 : 4);
        if (rc != QMS_OK) return rc;
        rc = check_device_ptr(d_offsets, "offsets", &dev2);
        if (rc != QMS_OK) return rc;
        if (d_vals) {
            rc = check_device_ptr(d_vals, "vals", &dev2);
            if (rc != QMS_OK) return rc;
        }
        DeviceScope scope(dev);
        std::vector<uint64_t> off(num_segments + 1);
        if (h_offsets) {
            for (uint32_t j = 0; j <= num_segments; ++j) off[j] = h_offsets[j];
        } else {
            hipError_t e = hipMemcpyAsync(off.data(), d_offsets, off.size() * sizeof(uint64_t),
                                          hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_error(e, "reading offsets");
        }
        if (off[0] != 0) return set_error(QMS_ERR_INVALID, "offsets[0] must be 0");
        for (uint32_t j = 0; j < num_segments; ++j)
            if (off[j + 1] < off[j]) return set_error(QMS_ERR_INVALID, "offsets decrease");
        for (uint32_t j = 0; j < num_segments; ++j)
            if (off[j + 1] - off[j] >= (1ull << 32))
                return set_error(QMS_ERR_UNSUPPORTED, "segment of 2^32 keys or more");
        WorkspaceLease ws;
        rc = get_workspace(dev, stream, &ws);
        if (rc != QMS_OK) return rc;
        // every round planned on the device: nothing is read back
        return sort_batch_device_rounds(dt, d_vals != nullptr, (char *)d_keys, d_vals, d_offsets,
                                        off.data(), num_segments, 0, *ws, stream);
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_sort_batch");
    }
}

extern "C" int qms_batch_check(hipStream_t stream) {
    try {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_error(e, "hipGetDevice");
        WorkspaceLease ws;
        int rc = get_workspace(dev, stream, &ws);
        if (rc != QMS_OK) return rc;
        uint32_t st[2] = {0, 0};
        const uint32_t zero[2] = {0, 0};
        e = hipMemcpyAsync(st, ws.get()->r_status, sizeof(st), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws.get()->r_status, zero, sizeof(zero), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_error(e, "reading the batch status");
        if (st[0] || st[1])
            return set_error(QMS_ERR_HIP, "a batch left " + std::to_string(st[1]) +
                                              " segments unsorted (" + std::to_string(st[0]) +
                                              " plan errors)");
        return QMS_OK;
    } catch (...) {
        return set_error(QMS_ERR_NOMEM, "host exception in qms_batch_check");
    }
}
