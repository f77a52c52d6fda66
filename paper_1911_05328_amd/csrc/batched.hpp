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
    int32_t kind;         // persistent kernel kind that runs it (0, 1, 2)
    int32_t tile;         // its tile edge
    // Packed operands (k-tiled 16-bit planes in the workspace, written by the
    // pack kernel at the start of every launch): A at ap (m x lp), B^T at bp
    // (n x lp); split precision adds lo planes at + a_plane / + b_plane.
    int32_t packed;
    int32_t overwrite;    // C = A B (plain stores) instead of C += A B
    int32_t pack_blocks;  // entries of the pack list for this problem
    int32_t reserved;
    const uint16_t* ap;
    const uint16_t* bp;
    int64_t lp, a_plane, b_plane;
};

struct BatchItem {
    uint32_t problem;  // index into the problem table
    uint32_t local;    // tile * split_k + slice
};

struct BatchCtl {
    uint32_t next;       // next work-list item of this queue to hand out
    uint32_t done;       // workgroups that have left (queue 0 of a kind counts them)
    uint32_t pack_next;  // next pack-list entry (queue 0 of the kind that packs)
    uint32_t error;      // set when a bounded wait for a problem's planes gave up
};

// Each kernel kind's work list is split into one queue per XCD: workgroup w
// drains queue w mod 8 first (its XCD under the round-robin dispatch), then
// takes what is left in the others.  Queue q holds items [begin[q],
// begin[q + 1]) of the kind's list.
constexpr int kBatchQueues = 8;
struct BatchQueues {
    uint32_t begin[kBatchQueues + 1];
};

// Persistent kernel kinds: 0 = 128 tiles staged from the caller's operands,
// 1 = 128 tiles over packed planes, 2 = 256 tiles over packed planes.
constexpr int kBatchKinds = 3;
int batched_tile();       // 128
// Whether the wide kind's launch packs the operands of this mode itself.
bool batched_fused_pack(int mode);
int batched_wide_tile();  // 256
// Resident workgroups of the persistent kernel of this kind.
// mode: 0 fp32 operands (BF16x3 split), 1 bf16 operands, 5 fp16 operands.
int batched_grid(int mode, int kind);
// One persistent launch over one work list (each kind has its own list and
// counter block).
// pack_list / npack / pack_done: when npack > 0 (one-plane modes, the kind
// launched first), the kernel first packs every entry of the pack list,
// counting finished blocks per problem in pack_done, and a tile waits for its
// problem's count; the last workgroup out resets the counts.
hipError_t launch_batched(int mode, int kind, int grid, const BatchProblem* probs, const BatchItem* items,
                          const BatchQueues& queues, BatchCtl* ctl, uint32_t* counters, float* temps,
                          hipStream_t st, const BatchItem* pack_list = nullptr, uint32_t npack = 0,
                          uint32_t* pack_done = nullptr, uint32_t nprob = 0);
// Pack every packed problem's operands, one workgroup per entry of the pack
// list (problem, block), a block being batched_pack_rows() plane rows x
// batched_pack_k() k of A (first) or B^T.
int batched_pack_rows();
int batched_pack_k();
hipError_t launch_batched_pack(int mode, const BatchProblem* probs, const BatchItem* list, int64_t blocks,
                               hipStream_t st);

}  // namespace starmm
