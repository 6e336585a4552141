// qms_host.hpp -- host helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "qms_internal.hpp"

namespace qms {

int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *where);
int check_device_ptr(const void *p, const char *what, int *device);
int get_workspace(int device, hipStream_t stream, Workspace **out);
int release_workspaces();

// One array [0, n) of keys (and payloads): the full QuickMergesort loop.
int sort_array(int dt, bool pairs, uint32_t *keys, uint32_t *vals, uint64_t n,
               const Workspace &ws, hipStream_t st, bool log);

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
