// qms_prof.cpp -- per-kernel-class event timing (see qms_prof.hpp).
#include "qms_prof.hpp"

#include <cstring>
#include <vector>

#include "qms.h"
#include "qms_host.hpp"

namespace qms {

namespace {
const char *kNames[K_NUM_CLASSES] = {"tile_sort", "merge_split", "merge", "part_count",
                                     "part_scan", "part_split", "part_swap"};

struct Rec {
    int cls;
    double bytes;
    hipEvent_t a, b;
};

struct ProfState {
    bool on = false;
    std::vector<hipEvent_t> pool;  // reusable events
    size_t used = 0;
    std::vector<Rec> recs;
    hipEvent_t take() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};
thread_local ProfState g_prof;
}  // namespace

bool prof_on() { return g_prof.on; }

void prof_start(hipStream_t st, int cls) {
    Rec r;
    r.cls = cls;
    r.bytes = 0;
    r.a = g_prof.take();
    r.b = g_prof.take();
    if (r.a) (void)hipEventRecord(r.a, st);
    g_prof.recs.push_back(r);
}

void prof_stop(hipStream_t st, int cls, double bytes) {
    for (auto it = g_prof.recs.rbegin(); it != g_prof.recs.rend(); ++it) {
        if (it->cls == cls) {
            it->bytes = bytes;
            if (it->b) (void)hipEventRecord(it->b, st);
            return;
        }
    }
}

}  // namespace qms

using namespace qms;

extern "C" {

int qms_profile_begin(void) {
    g_prof.on = true;
    g_prof.used = 0;
    g_prof.recs.clear();
    return QMS_OK;
}

int qms_profile_end(qms_kernel_stat *out, int max_entries, int *n_out) {
    g_prof.on = false;
    qms_kernel_stat acc[K_NUM_CLASSES];
    std::memset(acc, 0, sizeof(acc));
    for (int c = 0; c < K_NUM_CLASSES; ++c)
        std::strncpy(acc[c].name, kNames[c], sizeof(acc[c].name) - 1);
    int rc = QMS_OK;
    for (const Rec &r : g_prof.recs) {
        if (!r.a || !r.b) continue;
        hipError_t e = hipEventSynchronize(r.b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) {
            rc = hip_error(e, "qms_profile_end");
            break;
        }
        acc[r.cls].launches += 1;
        acc[r.cls].total_ms += ms;
        acc[r.cls].bytes += r.bytes;
    }
    g_prof.recs.clear();
    g_prof.used = 0;
    int n = 0;
    for (int c = 0; c < K_NUM_CLASSES && n < max_entries; ++c) {
        if (out) out[n] = acc[c];
        ++n;
    }
    if (n_out) *n_out = n;
    return rc;
}

}  // extern "C"
