// Tile core fed by direct global->LDS copies of k-tiled bf16 (or fp16) planes.
//
// A workgroup of NW waves computes a square BM x BN tile (BM = BN = 32 NW)
// from NPL planes per operand (1: one bf16 product; 2: hi/lo planes and the
// split-precision product Ah*Bl + Al*Bh + Ah*Bh), bf16 or (F16) fp16.  Each 16-deep k-stage
// (NPL planes x (BM + BN) rows x 32 bytes) is copied straight from global
// memory into one of S LDS stage buffers by global_load_lds_dwordx4, S-1
// stages ahead of the MFMAs.  In the k-tiled plane layout a 32-row x 16-k
// unit is 1 KB contiguous and already in LDS order, so each copy instruction
// moves one whole unit (64 lanes x 16 bytes) with no register staging; wave
// w copies row unit w of every plane of both operands.  A wave waits only for
// the stage it is about to read (partial vmcnt), and the MFMA fragments of
// stage s+1 are read into a second register set while the MFMAs of stage s
// run, one fragment read issued between MFMAs so MFMAs never queue behind
// all of a wave's LDS reads.  The stage buffers are separate LDS variables
// and the stage rotation is unrolled, so every access names its buffer at
// compile time; that lets the compiler keep the partial waits instead of
// draining all outstanding copies before each LDS read.
//
// Operand contract: planes 16-byte aligned, row length a multiple of 16 and
// >= ke rounded up to 16, zeros from k to the row length, rows padded to
// whole 32-row units.  Row units past m (n) are clamped to the last one, so
// they only feed outputs that are not stored.  MFMAs run in the same order
// as the staged core (tile_bf16.hpp), so results match it bitwise; the
// accumulator layout is Bf16Tile<BM, BN, WM, WN, *>'s.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "tile_bf16.hpp"

namespace starmm {

typedef __attribute__((address_space(3))) void* lds_void_ptr;

__device__ inline int64_t min_i64(int64_t a, int64_t b) { return a < b ? a : b; }

// s_waitcnt vmcnt(VM) lgkmcnt(0): gfx9 encoding vmcnt[3:0], expcnt[6:4],
// lgkmcnt[11:8], vmcnt[5:4] at [15:14]; expcnt left at its maximum.
template <int VM>
__device__ inline void wait_vm_lgkm0() {
    static_assert(VM >= 0 && VM < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((VM & 15) | (7 << 4) | ((VM >> 4) << 14));
}

// Wait with the vmcnt immediate chosen at run time from 0..MAX (each a
// compile-time wait).
template <int MAX>
__device__ inline void wait_vm_lgkm0_upto(int64_t vm) {
    if constexpr (MAX == 0) {
        wait_vm_lgkm0<0>();
    } else {
        if (vm >= MAX)
            wait_vm_lgkm0<MAX>();
        else
            wait_vm_lgkm0_upto<MAX - 1>(vm);
    }
}

// f(integral_constant<I>) for I = B .. E-1, unrolled at compile time.
template <int B, int E, class F>
__device__ inline void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Workgroup barrier that is also a compiler barrier for memory accesses but
// emits no wait of its own (the partial waits order the copies).
__device__ inline void stage_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Stage buffer I (BYTES bytes): one LDS variable per buffer, so the compiler
// can tell the buffers' copies apart when it places its waits.
template <int I, int BYTES>
__device__ inline uint8_t* dma_stage() {
    __shared__ __attribute__((aligned(1024))) uint8_t buf[BYTES];
    return buf;
}

template <int WM, int WN, int NPL, int S, bool F16 = false>
struct DmaTile {
    static constexpr int NW = WM * WN;
    static constexpr int BM = 32 * NW, BN = 32 * NW;
    static constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
    static constexpr int BK = kPlaneKBlock;                    // k per stage
    static constexpr int kStageBytes = NPL * (BM + BN) * 32;  // one unit row = 16 k x 2 bytes
    static constexpr int kCopies = 2 * NPL;                    // copies per wave per stage
    static constexpr int kReads = NPL * (FM + FN);             // fragment reads per wave per stage
    static constexpr int kMfma = (NPL == 2 ? 3 : 1) * FM * FN; // MFMAs per wave per stage
    static_assert(NPL == 1 || NPL == 2, "one or two planes");
    static_assert(S >= 3 && (int64_t)S * kStageBytes <= 160 * 1024, "stages must fit LDS");
    static_assert((S - 1) * kCopies < 64, "vmcnt range");

    // acc = A[row0:row0+BM, kb:ke] * B[kb:ke, col0:col0+BN] over planes A at
    // Ap (hi; lo at + a_plane), B^T at Bp (hi; lo at + b_plane), row lengths
    // lda / ldb.  All waves of the workgroup call it; returns with no copy in
    // flight.  The caller separates two calls by a workgroup barrier.
    __device__ static void compute(const uint16_t* Ap, int64_t lda, int64_t a_plane, const uint16_t* Bp, int64_t ldb,
                                   int64_t b_plane, int64_t m, int64_t n, int64_t row0, int64_t col0, int64_t kb,
                                   int64_t ke, f32x16 (&acc)[FM][FN]) {
        uint8_t* stages[S];
        static_for<0, S>([&](auto i) { stages[decltype(i)::value] = dma_stage<decltype(i)::value, kStageBytes>(); });

        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const int wm = wave / WN, wn = wave % WN;
        const int lrow = lane & 31, half = lane >> 5;

        // Copy side: wave w copies row unit w of each plane of both operands;
        // stage s is k-unit kb / 16 + s.  LDS stage layout: A planes, then B
        // planes, each BM (BN) rows of 32 bytes.
        const int64_t au = min_i64(row0 / 32 + wave, (m - 1) / 32), bu = min_i64(col0 / 32 + wave, (n - 1) / 32);
        const gptr<const uint16_t> ga = (gptr<const uint16_t>)Ap + au * 32 * lda + (kb / BK) * 512 + lane * 8;
        const gptr<const uint16_t> gb = (gptr<const uint16_t>)Bp + bu * 32 * ldb + (kb / BK) * 512 + lane * 8;
        auto issue = [&](uint8_t* stage, int64_t s) {
            const int64_t ko = s * 512;
            uint8_t* dst = stage + wave * 1024;
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
                __builtin_amdgcn_global_load_lds((const void*)(ga + p * a_plane + ko),
                                                 (lds_void_ptr)(dst + p * BM * 32), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((const void*)(gb + p * b_plane + ko),
                                                 (lds_void_ptr)(dst + (NPL * BM + p * BN) * 32), 16, 0, 0);
            }
        };

        // Read side: lane l reads row/col l%32 of each 32-row fragment, k-chunk l/32.
        const int roff = lrow * 32 + ((half ^ tiled_swz(lrow)) << 4);
        bf16x8 fa[2][NPL][FM], fb[2][NPL][FN];  // [register set][plane][fragment]
        auto read = [&](const uint8_t* stage, bf16x8 (&a)[NPL][FM], bf16x8 (&b)[NPL][FN]) {
#pragma unroll
            for (int p = 0; p < NPL; ++p) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    a[p][i] = *reinterpret_cast<const bf16x8*>(stage + p * BM * 32 + (wm * FM * 32 + i * 32) * 32 + roff);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[p][j] = *reinterpret_cast<const bf16x8*>(stage + (NPL * BM + p * BN) * 32 +
                                                              (wn * FN * 32 + j * 32) * 32 + roff);
            }
        };

#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
        auto mma = [&](const bf16x8 (&a)[NPL][FM], const bf16x8 (&b)[NPL][FN]) {
            if constexpr (NPL == 2) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mfma32x32x16<F16>(a[0][i], b[1][j], acc[i][j]);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mfma32x32x16<F16>(a[1][i], b[0][j], acc[i][j]);
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma32x32x16<F16>(a[0][i], b[0][j], acc[i][j]);
        };

        // MFMAs q in [QB, QE) of one stage in the order of mma(): product set
        // q / (FM FN) (lo x hi, hi x lo, hi x hi for two planes), then
        // fragment (i, j) = ((q % (FM FN)) / FN, q % FN).
        auto mma_range = [&](const bf16x8 (&a)[NPL][FM], const bf16x8 (&b)[NPL][FN], auto qb, auto qe) {
            static_for<decltype(qb)::value, decltype(qe)::value>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int set = q / (FM * FN), i = (q % (FM * FN)) / FN, j = q % FN;
                constexpr int pa = (NPL == 2 && set == 1) ? 1 : 0, pb = (NPL == 2 && set == 0) ? 1 : 0;
                acc[i][j] = mfma32x32x16<F16>(a[pa][i], b[pb][j], acc[i][j]);
            });
        };
        // MFMAs issued ahead of the stage barrier: they keep the matrix cores
        // busy while the waves meet there (they read registers only)
        constexpr int kPre = NPL == 2 ? FM * FN : (FM * FN) / 2;

        const int64_t nst = (ke - kb + BK - 1) / BK;
        // Stage kt's fragments sit in register set kt % 2.  Step kt: wait
        // until stage kt+1 has landed (copies of the stages issued after it
        // stay in flight), barrier, copy stage kt+S into the buffer stage kt
        // has left, read stage kt+1 into the other register set, then the
        // MFMAs of stage kt.  Steps are unrolled by lcm(S, 2) so buffer and
        // register set are compile-time.  Steady state (FULL): stage kt+S
        // exists, S-2 stages are in flight, and the step has no branch (a
        // skipped read on some path would make the MFMAs wait for every
        // outstanding LDS read).
        constexpr int U = S % 2 == 0 ? S : 2 * S;
        auto step = [&](int64_t kt, auto jtag, auto full_tag) {
            constexpr int J = decltype(jtag)::value;  // kt % U
            constexpr bool FULL = decltype(full_tag)::value;
            constexpr int buf = J % S, nbuf = (J + 1) % S, cur = J & 1, nxt = (J + 1) & 1;
            if (FULL) {
                mma_range(fa[cur], fb[cur], std::integral_constant<int, 0>{}, std::integral_constant<int, kPre>{});
                __builtin_amdgcn_sched_barrier(0);
                wait_vm_lgkm0<(S - 2) * kCopies>();
                stage_barrier();
                issue(stages[buf], kt + S);
                read(stages[nbuf], fa[nxt], fb[nxt]);
                mma_range(fa[cur], fb[cur], std::integral_constant<int, kPre>{}, std::integral_constant<int, kMfma>{});
                // issue order: the copies, then the fragment reads spread
                // evenly between the remaining MFMAs
                constexpr int kPost = kMfma - kPre;
                __builtin_amdgcn_sched_group_barrier(0x020, kCopies, 0);  // VMEM read: the copies
                static_for<0, kReads>([&](auto r) {
                    constexpr int R = decltype(r)::value;
                    constexpr int nm = kPost * (R + 1) / kReads - kPost * R / kReads;
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
                    if constexpr (nm > 0) __builtin_amdgcn_sched_group_barrier(0x008, nm, 0);  // MFMA
                });
                __builtin_amdgcn_sched_barrier(0);
                return;
            }
            if (kt + 1 < nst) {
                const int64_t last = kt + S - 1 < nst - 1 ? kt + S - 1 : nst - 1;  // last stage issued so far
                wait_vm_lgkm0_upto<(S - 2) * kCopies>((last - (kt + 1)) * kCopies);
                stage_barrier();
                if (kt + S < nst) issue(stages[buf], kt + S);
                read(stages[nbuf], fa[nxt], fb[nxt]);
            }
            mma(fa[cur], fb[cur]);
        };

        if (nst > 0) {
            static_for<0, S>([&](auto i) {
                constexpr int I = decltype(i)::value;
                if (I < nst) issue(stages[I], I);
            });
            // stage 0 landed: up to S-1 later stages in flight
            wait_vm_lgkm0_upto<(S - 1) * kCopies>((nst - 1 < S - 1 ? nst - 1 : S - 1) * kCopies);
            stage_barrier();
            read(stages[0], fa[0], fb[0]);
            int64_t kt = 0;
            for (; kt + U + S <= nst; kt += U)
                static_for<0, U>([&](auto j) { step(kt + decltype(j)::value, j, std::true_type{}); });
            for (; kt < nst; kt += U)  // at most (S + U) / U rounds
                static_for<0, U>([&](auto j) {
                    if (kt + decltype(j)::value < nst) step(kt + decltype(j)::value, j, std::false_type{});
                });
        }
        wait_vm_lgkm0<0>();  // no copy outlives the call
    }
};

}  // namespace starmm
