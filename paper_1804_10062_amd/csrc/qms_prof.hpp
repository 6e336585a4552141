// qms_prof.hpp -- optional per-kernel-class timing with HIP events on the
// launch stream, and the algorithmic bytes of each launch.
#pragma once

#include <hip/hip_runtime.h>

namespace qms {

enum KernelClass : int {
    K_TILE_SORT = 0,  // base case (LDS bitonic tile sort)
    K_MERGE_SPLIT,    // merge-path splits of a level
    K_MERGE,          // swap-merge of a level
    K_PART_COUNT,     // partition: per-tile class counts
    K_PART_SCAN,      // partition: scans (pass A, and pass B when it runs)
    K_PART_SPLIT,     // partition: chunk boundary positions
    K_PART_SWAP,      // partition: rank-matched exchange
    K_FINAL,          // the bitonic network of the loop's last ranges
    K_NUM_CLASSES
};

// True while the calling thread has profiling switched on.
bool prof_on();
// Record the start / end of one launch of class `cls` on stream `st`;
// `bytes` (end only) are the launch's algorithmic bytes; `level` tags a
// merge pass with the binary level it starts at (-1: none).
void prof_start(hipStream_t st, int cls, int level);
void prof_stop(hipStream_t st, int cls, double bytes);

// RAII helper around one launch.
struct ProfScope {
    hipStream_t st;
    int cls;
    double bytes;
    bool on;
    ProfScope(hipStream_t s, int c, double b, int level = -1)
        : st(s), cls(c), bytes(b), on(prof_on()) {
        if (on) prof_start(st, cls, level);
    }
    ~ProfScope() {
        if (on) prof_stop(st, cls, bytes);
    }
};

}  // namespace qms
