// Persistent batched kernel: one launch drains a work list of base-case
// output tiles drawn from many independent (+,x) products of uneven shape.
//
// Work distribution: the host sorts problems by descending cost
// (longest-processing-time first), cuts each problem's tiles, in the
// recursion's order, into chunks of the tiles one XCD holds at once, and
// deals the chunks to eight queues (one per XCD), least-loaded first.  A
// workgroup takes items from its own XCD's queue by that queue's device
// counter, then from the other queues in turn, so neighbouring tiles share
// an L2 and the tail of the launch is made of the cheapest items.  The last
// workgroup to leave resets the counters, so a captured graph of this
// single kernel can be replayed with no memset node.
//
// k-split per problem (s = 2^levels slices): every slice writes its partial
// tile to a workspace slot; the slice that arrives last at the tile's
// counter sums the s slots in ascending slice order and adds the sum to C.
// The result is therefore independent of which slice finishes last
// (deterministic), and each element of C is updated once per launch, by a
// no-return atomic add (the same bits as a load-add-store, without the wait).
//
// Packed problems (the default) first have their operands rewritten as
// k-tiled 16-bit planes (A and B^T, one plane for bf16 or fp16 inputs, bf16
// hi/lo for fp32), so every tile stages plain aligned 16-byte chunks
// whatever the caller's strides and alignment; unpacked problems stage
// straight from the caller's operands.  For bf16 / fp16 inputs the packing
// is the first phase of the persistent launch itself (a tile waits only for
// its own problem's blocks, so packing later problems overlaps the tiles of
// earlier ones); the fp32 split packs in a kernel of its own before it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "batched.hpp"
#include "internal.hpp"
#include "tile_bf16.hpp"
#include "tile_dma.hpp"

namespace starmm {

namespace {

constexpr int kBT = 128;  // batched tile edge (4 waves, 2 x 2)
// The in-launch pack phase (one-plane modes) is built but switched off: its
// first GPU run went silent past the harness's limit and no cause has been
// found by reading; the pack kernel runs before the launch instead.
#ifndef STARMM_FUSED_PACK
#define STARMM_FUSED_PACK 0
#endif

// Pointers read from the problem table are generic to the compiler, which
// would access them with flat instructions; flat loads also count against
// the LDS wait counter, so LDS waits would drain global traffic too.  Every
// table pointer is device global memory: access it as such.
template <class T>
__device__ inline gptr<T> as_global(T* p) {
    return (gptr<T>)p;
}

// Pack: one workgroup per block of 64 plane rows x 128 k of one operand of
// one problem (the pack list names the problem and the block; a problem's A
// blocks come before its B^T blocks).  The block is read with lanes along
// the operand's contiguous
// direction (k for A, columns for B), kept in LDS as [plane row][k], and
// written as its 2 x 4 units of 1 KB in tiled order; entries outside the
// operand are zeros.  SPLIT: fp32 operands -> hi/lo planes; else bf16 copy.
constexpr int kPackRows = 64, kPackK = 128;

// LDS image of one pack block: [plane row][k]; rows stay 16-byte aligned,
// offset by 16 bytes so neighbouring rows start in different banks.
template <bool SPLIT>
struct PackTile {
    using E = typename std::conditional<SPLIT, float, uint16_t>::type;
    static constexpr int VEC = 16 / (int)sizeof(E);  // elements per 16-byte load
    E t[kPackRows][kPackK + VEC];
};

// Pack block `it` with the NT threads of the workgroup (all of them call
// it); ends with the block's planes written (not yet visible to others).
template <bool SPLIT, int NT>
__device__ inline void pack_block(const BatchProblem* __restrict__ probs, const BatchItem it, PackTile<SPLIT>& pt) {
    using E = typename PackTile<SPLIT>::E;
    constexpr int VEC = PackTile<SPLIT>::VEC;
    auto& t = pt.t;
    const BatchProblem& p = probs[it.problem];
    const int64_t kblocks = (p.lp + kPackK - 1) / kPackK;
    const int64_t a_blocks = ((plane_rows_dev(p.m) + kPackRows - 1) / kPackRows) * kblocks;
    int64_t q = it.local;
    const bool is_b = q >= a_blocks;
    if (is_b) q -= a_blocks;
    const int64_t r0 = (q / kblocks) * kPackRows, k0 = (q % kblocks) * kPackK;
    const int64_t rows = is_b ? p.n : p.m;
    const gptr<const E> X = as_global(static_cast<const E*>(is_b ? p.B : p.A));
    // 16 bytes per lane along the operand's contiguous direction (A: k; B:
    // its columns = plane rows).  Whole in-range runs load as aligned 16-byte
    // blocks (load16_any never touches a block without a requested byte);
    // runs that cross the operand's edge go element by element.
    const int64_t cols = is_b ? p.n : p.k;       // extent of the contiguous direction
    const int64_t ld = is_b ? p.ldb : p.lda;
    for (int idx = threadIdx.x; idx < kPackRows * kPackK / VEC; idx += NT) {
        int64_t line, c0;  // source row (A row / B row = k) and first element of the run
        int lr, lk;        // LDS coordinates of the run's first element
        if (is_b) {
            const int kk = idx / (kPackRows / VEC), cc = (idx % (kPackRows / VEC)) * VEC;
            line = k0 + kk;
            c0 = r0 + cc;
            lr = cc;
            lk = kk;
        } else {
            const int rr = idx / (kPackK / VEC), kc = (idx % (kPackK / VEC)) * VEC;
            line = r0 + rr;
            c0 = k0 + kc;
            lr = rr;
            lk = kc;
        }
        const int64_t lines = is_b ? p.k : rows;
        E v[VEC];
        if (line < lines && c0 + VEC <= cols) {
            const uint4 w = load16_any(X + line * ld + c0);
            const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if constexpr (SPLIT)
                    v[e] = __builtin_bit_cast(float, ww[e]);
                else
                    v[e] = (uint16_t)(ww[e / 2] >> (16 * (e % 2)));
            }
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = (line < lines && c0 + e < cols) ? X[line * ld + c0 + e] : E(0);
        }
        if (is_b) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) t[lr + e][lk] = v[e];  // transpose into [plane row][k]
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) t[lr][lk + e] = v[e];
        }
    }
    __syncthreads();
    const int64_t prow_total = plane_rows_dev(rows);
    const gptr<uint16_t> dst = as_global(const_cast<uint16_t*>(is_b ? p.bp : p.ap));
    const int64_t lo_off = is_b ? p.b_plane : p.a_plane;
    constexpr int KU = kPackK / kPlaneKBlock;  // k units per block row
    for (int w = threadIdx.x; w < 2 * KU * 64; w += NT) {
        const int u = w >> 6, pp = w & 63;
        const int ub = u / KU, uk = u % KU;  // unit row block (of 2), k unit
        const int ri = pp >> 1, c = (pp & 1) ^ tiled_swz(ri);
        const int64_t prow = r0 + ub * kPlaneRowBlock + ri, kc = k0 + uk * kPlaneKBlock + c * 8;
        if (prow >= prow_total || kc >= p.lp) continue;
        const E* src = &t[ub * kPlaneRowBlock + ri][uk * kPlaneKBlock + c * 8];
        const int64_t off = tiled_off(prow, kc, p.lp);
        if constexpr (SPLIT) {
            uint4 vh, vl;
            split_pack8(src, vh, vl);
            *(gptr<u32x4>)(dst + off) = u32x4{vh.x, vh.y, vh.z, vh.w};
            *(gptr<u32x4>)(dst + lo_off + off) = u32x4{vl.x, vl.y, vl.z, vl.w};
        } else {
            *(gptr<u32x4>)(dst + off) = u32x4{src[0] | (uint32_t)src[1] << 16, src[2] | (uint32_t)src[3] << 16,
                                              src[4] | (uint32_t)src[5] << 16, src[6] | (uint32_t)src[7] << 16};
        }
    }
}

template <bool SPLIT>
__global__ void __launch_bounds__(256)
k_batched_pack(const BatchProblem* __restrict__ probs, const BatchItem* __restrict__ list) {
    __shared__ __attribute__((aligned(16))) PackTile<SPLIT> pt;
    pack_block<SPLIT, 256>(probs, list[blockIdx.x], pt);
}

// One instantiation per staging path (packed planes, or the caller's
// operands): a kernel holding both would carry the register needs of both.
// KIND 0: 128-wide tiles staged from the caller's operands (MODE 0 fp32
// split, 1 bf16) by the register-staged core.  KIND 1 / 2: 128- / 256-wide
// tiles over the packed planes by the direct-to-LDS core (hi/lo planes for
// MODE 0, one bf16 plane for MODE 1; 64 KB of stages per 128 tile, 128 KB
// per 256 tile).  One instantiation per kind: a kernel holding several cores
// would carry the register needs of all of them.
template <int KIND>
struct BatchKind {
    static constexpr int T = KIND == 2 ? 256 : 128;  // tile edge
    static constexpr int WM = KIND == 2 ? 4 : 2, WN = 2;
    static constexpr int NT = WM * WN * 64;
    static constexpr int PER_CU = KIND == 2 ? 1 : 2;  // resident workgroups the launch bound asks for
};

// Spins (s_sleep(8) steps, ~0.25 us each) of the bounded wait for a
// problem's planes: ~4 s, far beyond the whole pack phase.
constexpr uint64_t kPackSpinLimit = uint64_t(1) << 24;

template <int MODE, int KIND>
__global__ void __launch_bounds__(BatchKind<KIND>::NT, BatchKind<KIND>::PER_CU)
k_batched(const BatchProblem* __restrict__ probs, const BatchItem* __restrict__ items, BatchQueues qb,
          BatchCtl* __restrict__ ctl, uint32_t* __restrict__ counters, float* __restrict__ temps,
          const BatchItem* __restrict__ pack_list, uint32_t npack, uint32_t* __restrict__ pack_done,
          uint32_t nprob) {
    using K = BatchKind<KIND>;
    constexpr int T = K::T;
    using Tile = Bf16Tile<T, T, K::WM, K::WN, MODE>;  // staged core (KIND 0); accumulator layout of all
    using Dma = DmaTile<K::WM, K::WN, MODE == 0 ? 2 : 1, MODE == 0 ? 4 : 8, MODE == 5>;
    static_assert(Dma::BM == T && Dma::FM == Tile::FM && Dma::FN == Tile::FN, "same tile");
    constexpr int FM = Tile::FM, FN = Tile::FN, NT = Tile::NT;
    // the wide kind of the one-plane modes packs inside its launch (the fp32
    // split's pack tile would not fit beside the stage buffers, and the
    // 128-wide kind keeps two workgroups per CU without it)
    constexpr bool kFusedPack = KIND == 2 && MODE != 0 && STARMM_FUSED_PACK != 0;
    __shared__ uint32_t s_item;
    __shared__ int s_last;
    const int tid = threadIdx.x;

    // Pack phase: every workgroup takes pack-list entries by the shared
    // counter until none is left, then turns to the tiles.  A tile waits for
    // its problem's blocks only; every entry was handed to a running
    // workgroup (which waits for nothing) before any tile is taken, so every
    // wait ends (it is also bounded, with an error word).
    if constexpr (kFusedPack) {
        if (npack > 0) {
            __shared__ __attribute__((aligned(16))) PackTile<false> pt;
            for (;;) {
                if (tid == 0) s_item = atomicAdd(&ctl[0].pack_next, 1u);
                __syncthreads();
                const uint32_t pi = s_item;
                __syncthreads();
                if (pi >= npack) break;
                const BatchItem pit = pack_list[pi];
                pack_block<false, NT>(probs, pit, pt);
                // the block's planes visible device-wide, then counted (the
                // barrier also keeps the next block off the LDS image)
                __threadfence();
                __syncthreads();
                if (tid == 0) atomicAdd(&pack_done[pit.problem], 1u);
            }
        }
    }

    // own XCD's queue first, then the others in turn; each item is handed
    // out once by its queue's counter, and a workgroup leaves when all eight
    // queues are empty
    const int home = (int)(blockIdx.x & (kBatchQueues - 1));
    for (int qi = 0; qi < kBatchQueues; ++qi) {
    const int q = (home + qi) & (kBatchQueues - 1);
    const uint32_t qn = qb.begin[q + 1] - qb.begin[q];
    for (;;) {
        if (tid == 0) s_item = atomicAdd(&ctl[q].next, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= qn) break;

        const BatchItem it = items[qb.begin[q] + item];
        const BatchProblem& p = probs[it.problem];
        if constexpr (kFusedPack) {
            if (npack > 0 && p.packed) {
                // wait until this problem's planes are packed
                if (tid == 0) {
                    uint64_t spins = 0;
                    while (__hip_atomic_load(&pack_done[it.problem], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
                           (uint32_t)p.pack_blocks) {
                        if (++spins > kPackSpinLimit) {
                            atomicExch(&ctl[0].error, 1u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        const int64_t s = int64_t(1) << p.levels;
        const int64_t t = it.local / s;
        const int sigma = (int)(it.local % s);
        int64_t ti, tj;
        recursion_tile(t, p.tiles_m, p.tiles_n, &ti, &tj);
        const int64_t row0 = ti * T, col0 = tj * T;
        int64_t kb, ke;
        slice_k_range(sigma, p.levels, p.k, kBf16BK, &kb, &ke);

        f32x16 acc[FM][FN];
        // (both cores access their operands as global memory)
        if constexpr (KIND != 0) {
            Dma::compute(p.ap, p.lp, p.a_plane, p.bp, p.lp, p.b_plane, p.m, p.n, row0, col0, kb, ke, acc);
        } else {
            __shared__ __attribute__((aligned(16))) typename Tile::Smem sm;
            if (p.vec_ok)
                Tile::template compute<true>(sm, p.A, p.lda, p.B, p.ldb, p.m, p.n, row0, col0, kb, ke, 1, acc);
            else
                Tile::template compute<false>(sm, p.A, p.lda, p.B, p.ldb, p.m, p.n, row0, col0, kb, ke, 1, acc);
        }
        const gptr<float> Cg = as_global(p.C);

        if (p.levels > 0) {
            // Partial tile into this slice's slot, in register order (coalesced).
            const gptr<float> slot = as_global(temps) + p.temp_off + (t * s + sigma) * (int64_t)(T * T);
            // (one 32 x 32 accumulator block at a time: the scheduler would
            // otherwise keep every address of the tile live at once)
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) slot[((a * FN + b) * 16 + i) * NT + tid] = acc[a][b][i];
                    __builtin_amdgcn_sched_barrier(0);
                }
            __threadfence();
            __syncthreads();
            if (tid == 0) {
                const uint32_t prev = atomicAdd(&counters[p.counter_off + t], 1u);
                s_last = prev == (uint32_t)(s - 1);
            }
            __syncthreads();
            if (!s_last) continue;
            __threadfence();
            const gptr<const float> base = as_global(temps) + p.temp_off + t * s * (int64_t)(T * T);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc[a][b][i] = base[((a * FN + b) * 16 + i) * NT + tid];
                    __builtin_amdgcn_sched_barrier(0);
                }
            for (int64_t q = 1; q < s; ++q) {
                const gptr<const float> sl = base + q * (T * T);
#pragma unroll
                for (int a = 0; a < FM; ++a)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
#pragma unroll
                        for (int i = 0; i < 16; ++i) acc[a][b][i] += sl[((a * FN + b) * 16 + i) * NT + tid];
                        __builtin_amdgcn_sched_barrier(0);
                    }
            }
            if (tid == 0) counters[p.counter_off + t] = 0u;
        }
        if (p.overwrite) {
            // C = tile (MM_FLAG_OVERWRITE_C): plain stores, C is not read
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b) {
                    const int64_t gc = col0 + Tile::acc_col(b);
                    if (gc < p.n) {
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            const int64_t gr = row0 + Tile::acc_row(a, i);
                            if (gr < p.m) Cg[gr * p.ldc + gc] = acc[a][b][i];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            continue;
        }
        // C += tile: each element of C is updated once per launch (tiles and
        // problems are disjoint, split-K merged above), so a no-return atomic
        // add gives the bits a load-add-store would, without waiting for the
        // load: the workgroup moves on to its next item at once.
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                const int64_t gc = col0 + Tile::acc_col(b);
                if (gc < p.n) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int64_t gr = row0 + Tile::acc_row(a, i);
                        if (gr < p.m) __builtin_amdgcn_global_atomic_fadd_f32(Cg + gr * p.ldc + gc, acc[a][b][i]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
    }

    }

    // Leave: the last workgroup out resets the counters for the next launch.
    if (tid == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&ctl[0].done, 1u);
        if (prev == gridDim.x - 1) {
            for (int qq = 0; qq < kBatchQueues; ++qq) ctl[qq].next = 0u;
            ctl[0].done = 0u;
            if (npack > 0) {
                ctl[0].pack_next = 0u;
                for (uint32_t i = 0; i < nprob; ++i) pack_done[i] = 0u;
            }
            __threadfence();
        }
    }
}

}  // namespace

int batched_tile() { return kBT; }
bool batched_fused_pack(int mode) { return mode != 0 && STARMM_FUSED_PACK != 0; }
int batched_wide_tile() { return BatchKind<2>::T; }

template <int MODE, int KIND>
int grid_of(int cus) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batched<MODE, KIND>, BatchKind<KIND>::NT, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

template <int MODE>
int grid_of_kind(int kind, int cus) {
    return kind == 0 ? grid_of<MODE, 0>(cus) : (kind == 1 ? grid_of<MODE, 1>(cus) : grid_of<MODE, 2>(cus));
}

int batched_grid(int mode, int kind) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return mode == 0 ? grid_of_kind<0>(kind, cus) : (mode == 5 ? grid_of_kind<5>(kind, cus) : grid_of_kind<1>(kind, cus));
}

int batched_pack_rows() { return kPackRows; }
int batched_pack_k() { return kPackK; }

hipError_t launch_batched_pack(int mode, const BatchProblem* probs, const BatchItem* list, int64_t blocks,
                               hipStream_t st) {
    if (blocks == 0) return hipSuccess;
    if (blocks > (int64_t)UINT32_MAX) return hipErrorInvalidValue;
    ProfScope ps("batched_pack", st);
    const dim3 grid((unsigned)blocks);
    if (mode == 0)
        hipLaunchKernelGGL(k_batched_pack<true>, grid, dim3(256), 0, st, probs, list);
    else
        hipLaunchKernelGGL(k_batched_pack<false>, grid, dim3(256), 0, st, probs, list);
    return hipGetLastError();
}

template <int MODE>
void launch_kind(int kind, dim3 g, const BatchProblem* probs, const BatchItem* items, const BatchQueues& qb,
                 BatchCtl* ctl, uint32_t* counters, float* temps, hipStream_t st, const BatchItem* pack_list,
                 uint32_t npack, uint32_t* pack_done, uint32_t nprob) {
    if (kind == 0)
        hipLaunchKernelGGL((k_batched<MODE, 0>), g, dim3(BatchKind<0>::NT), 0, st, probs, items, qb, ctl, counters,
                           temps, pack_list, npack, pack_done, nprob);
    else if (kind == 1)
        hipLaunchKernelGGL((k_batched<MODE, 1>), g, dim3(BatchKind<1>::NT), 0, st, probs, items, qb, ctl, counters,
                           temps, pack_list, npack, pack_done, nprob);
    else
        hipLaunchKernelGGL((k_batched<MODE, 2>), g, dim3(BatchKind<2>::NT), 0, st, probs, items, qb, ctl, counters,
                           temps, pack_list, npack, pack_done, nprob);
}

hipError_t launch_batched(int mode, int kind, int grid, const BatchProblem* probs, const BatchItem* items,
                          const BatchQueues& queues, BatchCtl* ctl, uint32_t* counters, float* temps,
                          hipStream_t st, const BatchItem* pack_list, uint32_t npack, uint32_t* pack_done,
                          uint32_t nprob) {
    if ((queues.begin[kBatchQueues] == 0 && npack == 0) || grid == 0) return hipSuccess;
    if (mode != 0 && mode != 1 && mode != 5) return hipErrorInvalidValue;
    // only the one-plane modes' wide kind packs inside its launch
    if (npack > 0 && (mode == 0 || kind != 2 || !pack_list || !pack_done)) return hipErrorInvalidValue;
    ProfScope ps("batched", st);
    const dim3 g(grid);
    if (mode == 0)
        launch_kind<0>(kind, g, probs, items, queues, ctl, counters, temps, st, pack_list, npack, pack_done, nprob);
    else if (mode == 5)
        launch_kind<5>(kind, g, probs, items, queues, ctl, counters, temps, st, pack_list, npack, pack_done, nprob);
    else
        launch_kind<1>(kind, g, probs, items, queues, ctl, counters, temps, st, pack_list, npack, pack_done, nprob);
    return hipGetLastError();
}

}  // namespace starmm
