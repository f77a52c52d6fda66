// Persistent batched kernel: one launch drains a work list of base-case
// output tiles drawn from many independent (+,x) products of uneven shape.
//
// Work distribution: a device counter hands out list items in order; the
// host sorts the list by descending cost (longest-processing-time first),
// so the tail of the launch is made of the cheapest items.  The last
// workgroup to leave resets the counter, so a captured graph of this single
// kernel can be replayed with no memset node.
//
// k-split per problem (s = 2^levels slices): every slice writes its partial
// tile to a workspace slot; the slice that arrives last at the tile's
// counter sums the s slots in ascending slice order and adds the sum to C.
// The result is therefore independent of which slice finishes last
// (deterministic), and C is written once per tile.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batched.hpp"
#include "internal.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {

constexpr int kBT = 128;  // batched tile edge (4 waves, 2 x 2)

template <int MODE>
__global__ void __launch_bounds__(256, 2)
k_batched(const BatchProblem* __restrict__ probs, const BatchItem* __restrict__ items, int64_t total,
          BatchCtl* __restrict__ ctl, uint32_t* __restrict__ counters, float* __restrict__ temps) {
    using Tile = Bf16Tile<kBT, kBT, 2, 2, MODE>;
    constexpr int FM = Tile::FM, FN = Tile::FN, NT = Tile::NT;
    __shared__ __attribute__((aligned(16))) typename Tile::Smem sm;
    __shared__ uint32_t s_item;
    __shared__ int s_last;
    const int tid = threadIdx.x;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= total) break;

        const BatchItem it = items[item];
        const BatchProblem& p = probs[it.problem];
        const int64_t s = int64_t(1) << p.levels;
        const int64_t t = it.local / s;
        const int sigma = (int)(it.local % s);
        int64_t ti, tj;
        recursion_tile(t, p.tiles_m, p.tiles_n, &ti, &tj);
        const int64_t row0 = ti * kBT, col0 = tj * kBT;
        int64_t kb, ke;
        slice_k_range(sigma, p.levels, p.k, kBf16BK, &kb, &ke);

        f32x16 acc[FM][FN];
        if (p.vec_ok)
            Tile::template compute<true>(sm, p.A, p.lda, p.B, p.ldb, p.m, p.n, row0, col0, kb, ke, 1, acc);
        else
            Tile::template compute<false>(sm, p.A, p.lda, p.B, p.ldb, p.m, p.n, row0, col0, kb, ke, 1, acc);

        if (p.levels > 0) {
            // Partial tile into this slice's slot, in register order (coalesced).
            float* slot = temps + p.temp_off + (t * s + sigma) * (int64_t)(kBT * kBT);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
#pragma unroll
                    for (int i = 0; i < 16; ++i) slot[((a * FN + b) * 16 + i) * NT + tid] = acc[a][b][i];
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                const uint32_t prev = atomicAdd(&counters[p.counter_off + t], 1u);
                s_last = prev == (uint32_t)(s - 1);
            }
            __syncthreads();
            if (!s_last) continue;
            __threadfence();
            const float* base = temps + p.temp_off + t * s * (int64_t)(kBT * kBT);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc[a][b][i] = base[((a * FN + b) * 16 + i) * NT + tid];
            for (int64_t q = 1; q < s; ++q) {
                const float* sl = base + q * (kBT * kBT);
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b)
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[a][b][i] += sl[((a * FN + b) * 16 + i) * NT + tid];
            }
            if (tid == 0) counters[p.counter_off + t] = 0u;
        }
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                const int64_t gc = col0 + Tile::acc_col(b);
                if (gc >= p.n) continue;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int64_t gr = row0 + Tile::acc_row(a, i);
                    if (gr < p.m) p.C[gr * p.ldc + gc] += acc[a][b][i];
                }
            }
    }

    // Leave: the last workgroup out resets the counters for the next launch.
    if (tid == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&ctl->done, 1u);
        if (prev == gridDim.x - 1) {
            ctl->next = 0u;
            ctl->done = 0u;
            __threadfence();
        }
    }
}

}  // namespace

int batched_tile() { return kBT; }

int batched_grid(bool split3) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = split3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<0>, 256, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<1>, 256, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return cus * per_cu;
}

hipError_t launch_batched(bool split3, int grid, const BatchProblem* probs, const BatchItem* items, int64_t total,
                          BatchCtl* ctl, uint32_t* counters, float* temps, hipStream_t st) {
    if (total == 0 || grid == 0) return hipSuccess;
    ProfScope ps("batched", st);
    if (split3)
        hipLaunchKernelGGL(k_batched<0>, dim3(grid), dim3(256), 0, st, probs, items, total, ctl, counters, temps);
    else
        hipLaunchKernelGGL(k_batched<1>, dim3(grid), dim3(256), 0, st, probs, items, total, ctl, counters, temps);
    return hipGetLastError();
}

}  // namespace starmm
