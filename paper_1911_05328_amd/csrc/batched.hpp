// Device-side records of the persistent batched launch (built on the host,
// uploaded into the caller's workspace).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace starmm {

struct BatchProblem {
    int64_t m, n, k;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    float* C;
    int64_t ldc;
    int64_t tiles_m, tiles_n;
    int64_t temp_off;     // float offset of this problem's slice slots (split problems)
    int64_t counter_off;  // offset of its per-tile arrival counters
    int32_t levels;       // log2(split_k)
    int32_t vec_ok;
};

struct BatchItem {
    uint32_t problem;  // index into the problem table
    uint32_t local;    // tile * split_k + slice
};

struct BatchCtl {
    uint32_t next;  // next work-list item to hand out
    uint32_t done;  // workgroups that have left
};

int batched_tile();
int batched_grid(bool split3);
hipError_t launch_batched(bool split3, int grid, const BatchProblem* probs, const BatchItem* items, int64_t total,
                          BatchCtl* ctl, uint32_t* counters, float* temps, hipStream_t st);

}  // namespace starmm
