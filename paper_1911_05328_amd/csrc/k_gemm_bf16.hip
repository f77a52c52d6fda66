// (+,x) base-case tiles on bf16 MFMA (v_mfma_f32_32x32x16_bf16) with fp32
// accumulation.
//
//  MODE 0 (split precision): fp32 operands are split while they are staged
//    into LDS: hi = bf16(x), lo = bf16(x - hi), both round-to-nearest-even
//    (v_cvt_pk_bf16_f32).  The tile product is Ah*Bl + Al*Bh + Ah*Bh, the
//    two small terms issued first, all into one fp32 accumulator.
//  MODE 1: bf16 operands, one product (MODE 5: fp16 operands).
//  MODE 6 / 7: bf16 / fp16 operands copied once into one k-tiled plane each
//    (A, and B transposed), one product, by the direct-to-LDS tiles (256 or
//    128 wide).
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
#include "tile_dma.hpp"

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
    const bool unscale = sa.row_unscale != nullptr;
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int64_t gc = col0 + Tile::acc_col(b);
            if (gc >= n) continue;
            const float cu = unscale ? sa.col_unscale[gc] : 1.0f;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t gr = row0 + Tile::acc_row(a, i);
                if (gr >= m) continue;
                float* p = dst + gr * ldd + gc;
                // exact: the unscale factors are powers of two
                const float v = unscale ? acc[a][b][i] * (sa.row_unscale[gr] * cu) : acc[a][b][i];
                if (r_sar != 0 || sa.overwrite)
                    *p = v;
                else if (sa.atomic_c)
                    atomicAdd(p, v);
                else
                    *p += v;
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
    const int64_t per_product = tiles << sa.levels;
    int64_t logical = xcd_logical_id(blockIdx.x, (int64_t)gridDim.x);
    if (sa.batch > 1 && per_product % 8 == 0 && per_product >= 256) {
        // products of at least 256 workgroups: XCD x takes the x-th eighth
        // of every product in turn, so the XCDs read one product's operands
        // at a time (repeats across XCDs can then hit the memory-side
        // cache); an eighth is still a recursion-order block of the
        // product's tiles for the XCD's L2 (measured 0.6% faster for 7
        // products of 4096^3)
        const int64_t x = blockIdx.x & 7, q = blockIdx.x >> 3, per = per_product >> 3;
        logical = (q / per) * per_product + x * per + q % per;
    }
    if constexpr (BM == 256 && BN == 256) {
        // One product on 256 tiles, one workgroup per CU, 16 or 32 tiles
        // wide: each round of 256 workgroups covers whole bands of tile rows
        // (256 / tiles_n rows), and XCD x takes block (x mod 2, x div 2) of
        // the band cut 2 x 4 (8 x 4 or 4 x 8 tiles), so the XCDs share the
        // band's rows and repeat each other's misses (measured 1.7% faster
        // on an 8192^3 one-plane product)
        const int64_t band = tiles_n == 0 ? 0 : 256 / tiles_n;
        if (sa.batch == 1 && sa.levels == 0 && (tiles_n == 16 || tiles_n == 32) && tiles_m % band == 0) {
            const int64_t x = blockIdx.x & 7, q = blockIdx.x >> 3, r = q / 32, j = q % 32;
            const int64_t bw = tiles_n / 4, bh = band / 2;  // block: bh rows x bw columns
            const int64_t ti = r * band + (x & 1) * bh + j / bw, tj = (x >> 1) * bw + j % bw;
            t.bidx = 0;
            t.sigma = 0;
            t.row0 = ti * BM;
            t.col0 = tj * BN;
            slice_k_range(0, 0, k, sa.tk, &t.kb, &t.ke);
            return t;
        }
    }
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
    const size_t esz = MODE == 0 ? 4 : 2;  // fp32 operands (MODE 0) or bf16 / fp16 planes / operands
    const void* A = static_cast<const char*>(Av) + t.bidx * sa.stride_a * esz;
    const void* B = static_cast<const char*>(Bv) + t.bidx * sa.stride_b * esz;
    C += t.bidx * sa.stride_c;

    f32x16 acc[FM][FN];
    Tile::template compute<ALIGNED>(sm, A, lda, B, ldb, m, n, t.row0, t.col0, t.kb, t.ke, vec_ok, acc, sa.a_plane,
                                    sa.b_plane);
    store_acc<Tile>(acc, C, ldc, temps, t.bidx, t.sigma, m, n, t.row0, t.col0, sa);
}

// ---- 256 x 256 split-precision tile over k-tiled planes, fed by direct
// global->LDS copies (tile_dma.hpp): 8 waves (4 x 2, 64 x 128 each), three
// 32 KB stages of 16 k (A hi, A lo, B^T hi, B^T lo), two ahead of the MFMAs
// (three stages measured 0.7% faster than four, which matched five).
constexpr int kDmaWM = 4, kDmaWN = 2;
#ifndef STARMM_DMA_STAGES
#define STARMM_DMA_STAGES 3
#endif
template <bool F16>
using WideTile = DmaTile<kDmaWM, kDmaWN, 2, STARMM_DMA_STAGES, F16>;
constexpr int kDmaBM = WideTile<false>::BM, kDmaBN = WideTile<false>::BN, kDmaBK = WideTile<false>::BK;
constexpr int kDmaThreads = WideTile<false>::NW * 64;

// F16: fp16 hi/lo planes (fp16 MFMA); else bf16.
template <bool F16>
__global__ void __launch_bounds__(kDmaThreads)
k_bf16x3_dma(const uint16_t* __restrict__ Ap, int64_t lda, const uint16_t* __restrict__ Bp, int64_t ldb,
             float* __restrict__ C, int64_t ldc, float* __restrict__ temps, int64_t m, int64_t n, int64_t k,
             int64_t tiles_m, int64_t tiles_n, SliceArgs sa) {
    using Tile = Bf16Tile<kDmaBM, kDmaBN, kDmaWM, kDmaWN, 2>;  // accumulator layout
    const TileCoord t = tile_coord<kDmaBM, kDmaBN>(tiles_m, tiles_n, k, sa);
    f32x16 acc[WideTile<F16>::FM][WideTile<F16>::FN];
    WideTile<F16>::compute(Ap + t.bidx * sa.stride_a, lda, sa.a_plane, Bp + t.bidx * sa.stride_b, ldb, sa.b_plane, m,
                           n, t.row0, t.col0, t.kb, t.ke, acc);
    store_acc<Tile>(acc, C + t.bidx * sa.stride_c, ldc, temps, t.bidx, t.sigma, m, n, t.row0, t.col0, sa);
}

// ---- one-plane products (bf16 or fp16 inputs copied into k-tiled planes):
// the direct-to-LDS core with one plane per operand, 256 x 256 (8 waves) or
// 128 x 128 (4 waves), eight 16-deep stages (128 / 64 KB of LDS), seven in
// flight while the MFMAs of one run (32-deep stages of two k-units measured
// 1% faster here and 14% slower in the batched kernel, whose registers then
// spill, so not kept).
template <int WM, int WN, bool F16>
using PlaneTile = DmaTile<WM, WN, 1, 8, F16>;

template <int WM, int WN, bool F16>
__global__ void __launch_bounds__(WM * WN * 64)
k_bf16_planes_dma(const uint16_t* __restrict__ Ap, int64_t lda, const uint16_t* __restrict__ Bp, int64_t ldb,
                  float* __restrict__ C, int64_t ldc, float* __restrict__ temps, int64_t m, int64_t n, int64_t k,
                  int64_t tiles_m, int64_t tiles_n, SliceArgs sa) {
    using D = PlaneTile<WM, WN, F16>;
    using Tile = Bf16Tile<D::BM, D::BN, WM, WN, 2>;  // accumulator layout
    const TileCoord t = tile_coord<D::BM, D::BN>(tiles_m, tiles_n, k, sa);
    f32x16 acc[D::FM][D::FN];
    D::compute(Ap + t.bidx * sa.stride_a, lda, 0, Bp + t.bidx * sa.stride_b, ldb, 0, m, n, t.row0, t.col0, t.kb,
               t.ke, acc);
    store_acc<Tile>(acc, C + t.bidx * sa.stride_c, ldc, temps, t.bidx, t.sigma, m, n, t.row0, t.col0, sa);
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
    const bool planes_aligned = MODE < 2 || (sa.a_plane % 8 == 0 && sa.b_plane % 8 == 0);
    // Rows 16-byte aligned: plain vector loads; otherwise the funnel-shift path.
    const bool aligned = planes_aligned && (lda % align_elems == 0) && (ldb % align_elems == 0) && ((uintptr_t)A % 16 == 0) &&
                         ((uintptr_t)B % 16 == 0) && (sa.stride_a % align_elems == 0) &&
                         (sa.stride_b % align_elems == 0);
    const int vec_ok = 1;
    ProfScope ps(MODE == 1 || MODE == 6 ? "bf16_tile"
                 : (MODE == 5 || MODE == 7 ? "f16_tile" : (MODE == 4 ? "fp16x3_tile" : "bf16x3_tile")),
                 st);
    if constexpr (MODE == 6 || MODE == 7) {
        // one-plane products run on the direct-to-LDS tiles only
        const int64_t kr = round_up(k, kDmaBK);
        if constexpr (BM == BN && (BM == 256 || BM == 128)) {
            if (aligned && lda >= kr && ldb >= kr && lda % kDmaBK == 0 && ldb % kDmaBK == 0) {
                hipLaunchKernelGGL((k_bf16_planes_dma<WM, WN, MODE == 7>), dim3((unsigned)grid), dim3(WM * WN * 64),
                                   0, st, static_cast<const uint16_t*>(A), lda, static_cast<const uint16_t*>(B), ldb,
                                   C, ldc, temps, m, n, k, tiles_m, tiles_n, sa);
                return hipGetLastError();
            }
        }
        return hipErrorInvalidValue;
    } else {
    if constexpr ((MODE == 2 || MODE == 4) && BM == kDmaBM && BN == kDmaBN) {
        const int64_t kr = round_up(k, kDmaBK);
        if (aligned && lda >= kr && ldb >= kr && lda % kDmaBK == 0 && ldb % kDmaBK == 0) {
            hipLaunchKernelGGL(k_bf16x3_dma<MODE == 4>, dim3((unsigned)grid), dim3(kDmaThreads), 0, st,
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
    if (mode == 4) return launch_mode<4>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    if (mode == 5) return launch_mode<5>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    if (mode == 6) return launch_mode<6>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    if (mode == 7) return launch_mode<7>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    return launch_mode<2>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
}

}  // namespace starmm
