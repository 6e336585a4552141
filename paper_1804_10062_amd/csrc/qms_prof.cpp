// qms_prof.cpp -- per-kernel-class event timing (see qms_prof.hpp).
#include "qms_prof.hpp"

#include <cstdio>
#include <cstring>
#include <vector>

#include "qms.h"
#include "qms_host.hpp"

namespace qms {

namespace {
const char *kNames[K_NUM_CLASSES] = {"tile_sort", "merge_split", "merge", "part_count",
                                     "part_scan", "part_split", "part_swap", "final_x"};

struct Rec {
    int cls;
    int level;  // merge passes: the binary level the pass starts at
    double bytes;
    hipEvent_t a, b;
};
constexpr int kMaxProfLevels = 32;

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

void prof_start(hipStream_t st, int cls, int level) {
    Rec r;
    r.cls = cls;
    r.level = level;
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
    qms_kernel_stat lev[kMaxProfLevels];
    std::memset(acc, 0, sizeof(acc));
    std::memset(lev, 0, sizeof(lev));
    for (int c = 0; c < K_NUM_CLASSES; ++c)
        std::strncpy(acc[c].name, kNames[c], sizeof(acc[c].name) - 1);
    for (int l = 0; l < kMaxProfLevels; ++l)
        std::snprintf(lev[l].name, sizeof(lev[l].name), "merge_level_%d", l);
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
        if (r.cls == K_MERGE && r.level >= 0 && r.level < kMaxProfLevels) {
            lev[r.level].launches += 1;
            lev[r.level].total_ms += ms;
            lev[r.level].bytes += r.bytes;
        }
    }
    g_prof.recs.clear();
    g_prof.used = 0;
    int n = 0;
    for (int c = 0; c < K_NUM_CLASSES && n < max_entries; ++c) {
        if (out) out[n] = acc[c];
        ++n;
    }
    // then the swap-merge passes by the level they start at
    for (int l = 0; l < kMaxProfLevels && n < max_entries; ++l) {
        if (lev[l].launches == 0) continue;
        if (out) out[n] = lev[l];
        ++n;
    }
    if (n_out) *n_out = n;
    return rc;
}

}  // extern "C"
