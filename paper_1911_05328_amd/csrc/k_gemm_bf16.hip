// (+,x) base-case tiles on bf16 MFMA (v_mfma_f32_32x32x16_bf16) with fp32
// accumulation.
//
//  MODE 0 (split precision): fp32 operands are split while they are staged
//    into LDS: hi = bf16(x), lo = bf16(x - hi), both round-to-nearest-even
//    (v_cvt_pk_bf16_f32).  The tile product is Ah*Bl + Al*Bh + Ah*Bh, the
//    two small terms issued first, all into one fp32 accumulator.
//  MODE 1: bf16 operands, one product.
//
// LDS holds both operands k-contiguous ([row][k] for A, [col][k] for B, rows
// padded to 80 bytes so 16-byte reads of 32 consecutive rows are
// conflict-free).  MFMA lane layout (32x32x16): lane l supplies row/col l%32
// and the 8 consecutive k values 8*(l/32)..+7 of the 16-deep step;
// accumulator register i of lane l is C[8*(i/4) + 4*(l/32) + i%4][l%32].
//
// The grid flattens (product, k-slice, output tile) exactly as the fp32 and
// semiring kernels do: tiles in recursion order, XCD-aware numbering.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "kcommon.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {





// Slice-0 results go to C (+= or atomically, or = when overwriting); other
// SAR slices write their own temporary.  Tile::acc_row/acc_col give the
// accumulator layout.
template <class Tile, int FM, int FN>
__device__ inline void store_acc(const f32x16 (&acc)[FM][FN], float* __restrict__ C, int64_t ldc,
                                 float* __restrict__ temps, int64_t bidx, int sigma, int64_t m, int64_t n,
                                 int64_t row0, int64_t col0, const SliceArgs& sa) {
    const int r_sar = sigma & ((1 << sa.sar_levels) - 1);
    const int g_tar = sigma >> sa.sar_levels;
    const int per_group = (1 << sa.sar_levels) - 1;
    float* dst;
    int64_t ldd;
    if (r_sar == 0) {
        dst = C;
        ldd = ldc;
    } else {
        dst = temps + bidx * sa.temp_batch_stride + (int64_t)(g_tar * per_group + r_sar - 1) * sa.temp_stride;
        ldd = sa.ldt;
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int64_t gc = col0 + Tile::acc_col(b);
            if (gc >= n) continue;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t gr = row0 + Tile::acc_row(a, i);
                if (gr >= m) continue;
                float* p = dst + gr * ldd + gc;
                if (r_sar != 0 || sa.overwrite)
                    *p = acc[a][b][i];
                else if (sa.atomic_c)
                    atomicAdd(p, acc[a][b][i]);
                else
                    *p += acc[a][b][i];
            }
        }
}

// Workgroup -> (product, k-slice, output tile): tiles in recursion order,
// XCD-aware numbering.
struct TileCoord {
    int64_t bidx, row0, col0, kb, ke;
    int sigma;
};

template <int BM, int BN>
__device__ inline TileCoord tile_coord(int64_t tiles_m, int64_t tiles_n, int64_t k, const SliceArgs& sa) {
    TileCoord t;
    const int64_t tiles = tiles_m * tiles_n;
    const int64_t logical = xcd_logical_id(blockIdx.x, (int64_t)gridDim.x);
    const int64_t per_product = tiles << sa.levels;
    t.bidx = logical / per_product;
    const int64_t rem = logical % per_product;
    t.sigma = (int)(rem / tiles);
    int64_t ti, tj;
    recursion_tile(rem % tiles, tiles_m, tiles_n, &ti, &tj);
    t.row0 = ti * BM;
    t.col0 = tj * BN;
    slice_k_range(t.sigma, sa.levels, k, sa.tk, &t.kb, &t.ke);
    return t;
}

template <int BM, int BN, int WM, int WN, int MODE, bool ALIGNED>
__global__ void __launch_bounds__(WM * WN * 64)
k_bf16_tile(const void* __restrict__ Av, int64_t lda, const void* __restrict__ Bv, int64_t ldb,
            float* __restrict__ C, int64_t ldc, float* __restrict__ temps, int64_t m, int64_t n, int64_t k,
            int64_t tiles_m, int64_t tiles_n, SliceArgs sa, int vec_ok) {
    using Tile = Bf16Tile<BM, BN, WM, WN, MODE>;
    constexpr int FM = Tile::FM, FN = Tile::FN;
    __shared__ __attribute__((aligned(16))) typename Tile::Smem sm;

    const TileCoord t = tile_coord<BM, BN>(tiles_m, tiles_n, k, sa);
    const size_t esz = MODE == 0 ? 4 : 2;  // fp32 operands (MODE 0) or bf16 planes / operands
    const void* A = static_cast<const char*>(Av) + t.bidx * sa.stride_a * esz;
    const void* B = static_cast<const char*>(Bv) + t.bidx * sa.stride_b * esz;
    C += t.bidx * sa.stride_c;

    f32x16 acc[FM][FN];
    Tile::template compute<ALIGNED>(sm, A, lda, B, ldb, m, n, t.row0, t.col0, t.kb, t.ke, vec_ok, acc, sa.a_plane,
                                    sa.b_plane);
    store_acc<Tile>(acc, C, ldc, temps, t.bidx, t.sigma, m, n, t.row0, t.col0, sa);
}

// ---- 256 x 256 tile over pre-split k-tiled planes, fed by direct
// global->LDS loads.
//
// Each 16-deep k-stage (A hi, A lo, B^T hi, B^T lo: 4 x 256 rows x 32 bytes
// = 32 KB) is copied straight from global memory into one of four LDS stage
// buffers by global_load_lds_dwordx4, three stages ahead of the MFMAs.  In
// the k-tiled plane layout a 32-row x 16-k unit is 1 KB contiguous and
// already in LDS order, so each copy instruction moves one whole unit (64
// lanes x 16 bytes) with no register staging.  A wave waits only for the
// stage it is about to read (partial vmcnt), and the MFMA fragments of stage
// s+1 are read into a second register set while the MFMAs of stage s run.
// The four buffers are separate LDS variables and the stage rotation is
// unrolled, so every access names its buffer at compile time; that lets the
// compiler keep the partial waits instead of draining all outstanding copies
// before each LDS read.
//
// Operand contract (checked on the host where it can be): planes 16-byte
// aligned, row length a multiple of 16 and >= k rounded up to 16, columns
// [k, row length) zero, rows padded to whole 32-row units, so a ragged last
// stage reads zeros.  Row units past m (n) are clamped to the last one, so
// they only feed outputs that are not stored.  MFMAs run in the same order
// as the staged kernel, so results match it bitwise.
constexpr int kDmaBM = 256, kDmaBN = 256, kDmaWM = 4, kDmaWN = 2;
constexpr int kDmaThreads = kDmaWM * kDmaWN * 64;
constexpr int kDmaBK = 16;
constexpr int kDmaStageBytes = (2 * kDmaBM + 2 * kDmaBN) * kDmaBK * 2;
#ifndef STARMM_DMA_STAGES
#define STARMM_DMA_STAGES 4
#endif
constexpr int kDmaStages = STARMM_DMA_STAGES;  // stage buffers (LDS: kDmaStages x 32 KB)
static_assert(kDmaStages >= 3 && kDmaStages * kDmaStageBytes <= 160 * 1024, "stages must fit LDS");
constexpr int kDmaPerWave = kDmaStageBytes / 1024 / (kDmaThreads / 64);  // copies per wave per stage

typedef __attribute__((address_space(3))) void* lds_void_ptr;

__device__ inline int64_t min_i64(int64_t a, int64_t b) { return a < b ? a : b; }

// s_waitcnt vmcnt(VM) lgkmcnt(0): gfx9 encoding vmcnt[3:0], expcnt[6:4],
// lgkmcnt[11:8], vmcnt[5:4] at [15:14]; expcnt left at its maximum.
template <int VM>
__device__ inline void wait_vm_lgkm0() {
    static_assert(VM >= 0 && VM < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((VM & 15) | (7 << 4) | ((VM >> 4) << 14));
}

// Stage buffer I of the wide tile: one LDS variable per buffer, so the
// compiler can tell the buffers' copies apart when it places its waits.
template <int I>
__device__ inline uint8_t* dma_stage() {
    __shared__ __attribute__((aligned(1024))) uint8_t buf[kDmaStageBytes];
    return buf;
}

// f(integral_constant<I>) for I = B .. E-1, unrolled at compile time.
template <int B, int E, class F>
__device__ inline void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
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

// Workgroup barrier that is also a compiler barrier for memory accesses but
// emits no wait of its own (the partial waits above order the copies).
__device__ inline void stage_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__global__ void __launch_bounds__(kDmaThreads)
k_bf16x3_dma(const uint16_t* __restrict__ Ap, int64_t lda, const uint16_t* __restrict__ Bp, int64_t ldb,
             float* __restrict__ C, int64_t ldc, float* __restrict__ temps, int64_t m, int64_t n, int64_t k,
             int64_t tiles_m, int64_t tiles_n, SliceArgs sa) {
    using Tile = Bf16Tile<kDmaBM, kDmaBN, kDmaWM, kDmaWN, 2>;  // accumulator layout only
    constexpr int FM = Tile::FM, FN = Tile::FN;
    constexpr int S = kDmaStages;
    uint8_t* stages[S];
    static_for<0, S>([&](auto i) { stages[decltype(i)::value] = dma_stage<decltype(i)::value>(); });

    const TileCoord t = tile_coord<kDmaBM, kDmaBN>(tiles_m, tiles_n, k, sa);
    Ap += t.bidx * sa.stride_a;
    Bp += t.bidx * sa.stride_b;
    C += t.bidx * sa.stride_c;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave / kDmaWN, wn = wave % kDmaWN;
    const int lrow = lane & 31, half = lane >> 5;

    // Copy side: wave w copies row unit w of the tile (rows 32w..32w+31) of
    // each of the four planes; stage s is k-unit kb / 16 + s.
    const int64_t au = min_i64(t.row0 / 32 + wave, (m - 1) / 32), bu = min_i64(t.col0 / 32 + wave, (n - 1) / 32);
    const uint16_t* ga = Ap + au * 32 * lda + (t.kb / kDmaBK) * 512 + lane * 8;
    const uint16_t* gb = Bp + bu * 32 * ldb + (t.kb / kDmaBK) * 512 + lane * 8;
    auto issue = [&](uint8_t* stage, int64_t s) {
        const int64_t ko = s * 512;
        uint8_t* dst = stage + wave * 1024;
        __builtin_amdgcn_global_load_lds(ga + ko, (lds_void_ptr)(dst), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(ga + sa.a_plane + ko, (lds_void_ptr)(dst + kDmaBM * 32), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(gb + ko, (lds_void_ptr)(dst + 2 * kDmaBM * 32), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(gb + sa.b_plane + ko, (lds_void_ptr)(dst + 2 * kDmaBM * 32 + kDmaBN * 32),
                                         16, 0, 0);
    };
    static_assert(kDmaPerWave == 4, "one copy per plane per wave");

    // Read side: lane l reads row/col l%32 of each 32-row fragment, k-chunk l/32.
    const int roff = lrow * 32 + ((half ^ tiled_swz(lrow)) << 4);
    bf16x8 fa[2][2][FM], fb[2][2][FN];  // [register set][plane][fragment]
    auto read = [&](const uint8_t* stage, bf16x8 (&a)[2][FM], bf16x8 (&b)[2][FN]) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[p][i] = *reinterpret_cast<const bf16x8*>(stage + p * kDmaBM * 32 + (wm * FM * 32 + i * 32) * 32 + roff);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                b[p][j] = *reinterpret_cast<const bf16x8*>(stage + (2 * kDmaBM + p * kDmaBN) * 32 +
                                                          (wn * FN * 32 + j * 32) * 32 + roff);
        }
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;
    auto mma = [&](const bf16x8 (&a)[2][FM], const bf16x8 (&b)[2][FN]) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
    };

    const int64_t nst = (t.ke - t.kb + kDmaBK - 1) / kDmaBK;
    // Stage kt's fragments sit in register set kt % 2.  Step kt: wait until
    // stage kt+1 has landed (the copies of the stages issued after it stay
    // in flight), barrier, copy stage kt+S into the buffer stage kt has left,
    // read stage kt+1 into the other register set, then the MFMAs of stage
    // kt.  Steps are unrolled by lcm(S, 2) so buffer and register set are
    // compile-time.  Steady state (FULL): stage kt+S exists, S-2 stages are
    // in flight, and the step has no branch (a skipped read on some path
    // would make the MFMAs wait for every outstanding LDS read).
    constexpr int U = S % 2 == 0 ? S : 2 * S;
    auto step = [&](int64_t kt, auto jtag, auto full_tag) {
        constexpr int J = decltype(jtag)::value;  // kt % U
        constexpr bool FULL = decltype(full_tag)::value;
        constexpr int buf = J % S, nbuf = (J + 1) % S, cur = J & 1, nxt = (J + 1) & 1;
        if (FULL) {
            wait_vm_lgkm0<(S - 2) * kDmaPerWave>();
            stage_barrier();
            issue(stages[buf], kt + S);
            read(stages[nbuf], fa[nxt], fb[nxt]);
            mma(fa[cur], fb[cur]);
            // Issue order: the copies, then one fragment read per two MFMAs,
            // so a wave's MFMAs never queue behind all of its LDS reads.
            __builtin_amdgcn_sched_group_barrier(0x020, kDmaPerWave, 0);  // VMEM read: the copies
#pragma unroll
            for (int r = 0; r < 2 * (FM + FN); ++r) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // DS read
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // MFMA
            }
            __builtin_amdgcn_sched_barrier(0);
            return;
        }
        if (kt + 1 < nst) {
            const int64_t last = kt + S - 1 < nst - 1 ? kt + S - 1 : nst - 1;  // last stage issued so far
            wait_vm_lgkm0_upto<(S - 2) * kDmaPerWave>((last - (kt + 1)) * kDmaPerWave);
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
        wait_vm_lgkm0_upto<(S - 1) * kDmaPerWave>((nst - 1 < S - 1 ? nst - 1 : S - 1) * kDmaPerWave);
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
    wait_vm_lgkm0<0>();  // no copy outlives the workgroup
    store_acc<Tile>(acc, C, ldc, temps, t.bidx, t.sigma, m, n, t.row0, t.col0, sa);
}

template <int BM, int BN, int WM, int WN, int MODE>
hipError_t launch_cfg(const Plan& p, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                      int64_t ldb, float* C, int64_t ldc, float* temps, const SliceArgs& sa_in, hipStream_t st) {
    const mm_plan_info& pi = p.info;
    SliceArgs sa = sa_in;
    sa.levels = pi.tar_levels + pi.sar_levels;
    sa.sar_levels = pi.sar_levels;
    sa.tk = kBf16BK;
    sa.atomic_c = pi.tar_levels > 0;
    sa.temp_stride = p.temp_stride;
    sa.ldt = p.ldt;
    const int64_t tiles_m = ceil_div(m, BM), tiles_n = ceil_div(n, BN);
    const int64_t grid = tiles_m * tiles_n * pi.sched.split_k * sa.batch;
    if (grid == 0) return hipSuccess;
    const int64_t align_elems = MODE == 0 ? 4 : 8;
    const bool planes_aligned = MODE != 2 || (sa.a_plane % 8 == 0 && sa.b_plane % 8 == 0);
    // Rows 16-byte aligned: plain vector loads; otherwise the funnel-shift path.
    const bool aligned = planes_aligned && (lda % align_elems == 0) && (ldb % align_elems == 0) && ((uintptr_t)A % 16 == 0) &&
                         ((uintptr_t)B % 16 == 0) && (sa.stride_a % align_elems == 0) &&
                         (sa.stride_b % align_elems == 0);
    const int vec_ok = 1;
    ProfScope ps(MODE == 1 ? "bf16_tile" : "bf16x3_tile", st);
    if constexpr (MODE == 2 && BM == kDmaBM && BN == kDmaBN) {
        const int64_t kr = round_up(k, kDmaBK);
        if (aligned && lda >= kr && ldb >= kr && lda % kDmaBK == 0 && ldb % kDmaBK == 0) {
            hipLaunchKernelGGL(k_bf16x3_dma, dim3((unsigned)grid), dim3(kDmaThreads), 0, st,
                               static_cast<const uint16_t*>(A), lda, static_cast<const uint16_t*>(B), ldb, C, ldc,
                               temps, m, n, k, tiles_m, tiles_n, sa);
            return hipGetLastError();
        }
    }
    if (aligned)
        hipLaunchKernelGGL((k_bf16_tile<BM, BN, WM, WN, MODE, true>), dim3((unsigned)grid), dim3(WM * WN * 64), 0, st,
                           A, lda, B, ldb, C, ldc, temps, m, n, k, tiles_m, tiles_n, sa, vec_ok);
    else
        hipLaunchKernelGGL((k_bf16_tile<BM, BN, WM, WN, MODE, false>), dim3((unsigned)grid), dim3(WM * WN * 64), 0,
                           st, A, lda, B, ldb, C, ldc, temps, m, n, k, tiles_m, tiles_n, sa, vec_ok);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const Plan& p, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                       int64_t ldb, float* C, int64_t ldc, float* temps, const SliceArgs& sa, hipStream_t st) {
    switch (p.info.sched.tile) {
        case 256: return launch_cfg<256, 256, 4, 2, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
        case 128: return launch_cfg<128, 128, 2, 2, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
        case 64: return launch_cfg<64, 64, 2, 2, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
        default: return launch_cfg<32, 32, 1, 1, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
    }
}

}  // namespace

hipError_t launch_bf16_tiles(const Plan& p, int mode, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                             const void* B, int64_t ldb, float* C, int64_t ldc, float* temps, int64_t band_row0,
                             int64_t band_m, const SliceArgs& sa, hipStream_t st) {
    (void)m;
    const size_t esz = mode == 0 ? 4 : 2;
    const void* Ab = static_cast<const char*>(A) + band_row0 * lda * esz;
    float* Cb = C + band_row0 * ldc;
    if (mode == 0) return launch_mode<0>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    if (mode == 1) return launch_mode<1>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    return launch_mode<2>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
}

}  // namespace starmm
