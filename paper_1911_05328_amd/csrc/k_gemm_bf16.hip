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

namespace starmm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBK = 32;    // k per staged tile
constexpr int kLd = kBK + 8;  // LDS row stride in bf16 elements (80 bytes)

__device__ inline uint32_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf16_value(uint32_t bits) { return __builtin_bit_cast(float, bits << 16); }

// Split x into hi/lo bf16 bit patterns (RNE each).
__device__ inline void split2(float x, uint32_t& hi, uint32_t& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

template <int BM, int BN, int WM, int WN, int MODE>
__global__ void __launch_bounds__(WM * WN * 64)
k_bf16_tile(const void* __restrict__ Av, int64_t lda, const void* __restrict__ Bv, int64_t ldb,
            float* __restrict__ C, int64_t ldc, float* __restrict__ temps, int64_t m, int64_t n, int64_t k,
            int64_t tiles_m, int64_t tiles_n, SliceArgs sa, int vec_ok) {
    constexpr int NT = WM * WN * 64;
    constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
    constexpr int NP = MODE == 0 ? 2 : 1;  // planes per operand (hi, lo)
    static_assert(FM >= 1 && FN >= 1, "bad tile");

    __shared__ __attribute__((aligned(16))) uint16_t As[2][NP][BM][kLd];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NP][BN][kLd];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int lrow = lane & 31, half = lane >> 5;

    const int64_t tiles = tiles_m * tiles_n;
    const int64_t logical = xcd_logical_id(blockIdx.x, (int64_t)gridDim.x);
    const int64_t per_product = tiles << sa.levels;
    const int64_t bidx = logical / per_product;
    const int64_t rem = logical % per_product;
    const int sigma = (int)(rem / tiles);
    int64_t ti, tj;
    recursion_tile(rem % tiles, tiles_m, tiles_n, &ti, &tj);
    const int64_t row0 = ti * BM, col0 = tj * BN;
    int64_t kb, ke;
    slice_k_range(sigma, sa.levels, k, sa.tk, &kb, &ke);

    const float* Af = reinterpret_cast<const float*>(Av) + bidx * sa.stride_a;
    const float* Bf = reinterpret_cast<const float*>(Bv) + bidx * sa.stride_b;
    const uint16_t* Ah = reinterpret_cast<const uint16_t*>(Av) + bidx * sa.stride_a;
    const uint16_t* Bh = reinterpret_cast<const uint16_t*>(Bv) + bidx * sa.stride_b;
    C += bidx * sa.stride_c;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

    const bool rows_full = row0 + BM <= m;
    const bool cols_full = col0 + BN <= n;

    // ---- staging registers
    // MODE 0: A as float4 chunks (4 k of one row); B as pairs of float4
    //         (rows k, k+1; 4 columns), packed into k-pair words in LDS.
    // MODE 1: A as 8-bf16 chunks; B as pairs of 8-bf16 rows.
    constexpr int AW = MODE == 0 ? 4 : 8;  // elements per A chunk
    constexpr int BW = MODE == 0 ? 4 : 8;  // columns per B pair
    constexpr int A_TOT = BM * kBK / AW, B_TOT = BN * kBK / (2 * BW);
    constexpr int A_CH = (A_TOT + NT - 1) / NT, B_CH = (B_TOT + NT - 1) / NT;
    float ra[MODE == 0 ? A_CH : 1][4];
    float rb[MODE == 0 ? B_CH : 1][2][4];
    uint4 ha[MODE == 1 ? A_CH : 1];
    uint4 hb[MODE == 1 ? B_CH : 1][2];

    auto load_tiles = [&](int64_t k0) {
        const bool k_full = k0 + kBK <= ke;
#pragma unroll
        for (int c = 0; c < A_CH; ++c) {
            const int idx = tid + c * NT;
            if (A_TOT % NT != 0 && idx >= A_TOT) break;
            const int r = idx / (kBK / AW), kc = (idx % (kBK / AW)) * AW;
            const int64_t gr = row0 + r, gk = k0 + kc;
            const bool fast = vec_ok && k_full && (rows_full || gr < m);
            if constexpr (MODE == 0) {
                if (fast) {
                    const float4 v = *reinterpret_cast<const float4*>(Af + gr * lda + gk);
                    ra[c][0] = v.x; ra[c][1] = v.y; ra[c][2] = v.z; ra[c][3] = v.w;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) ra[c][e] = (gr < m && gk + e < ke) ? Af[gr * lda + gk + e] : 0.0f;
                }
            } else {
                if (fast) {
                    ha[c] = *reinterpret_cast<const uint4*>(Ah + gr * lda + gk);
                } else {
                    uint16_t v[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = (gr < m && gk + e < ke) ? Ah[gr * lda + gk + e] : (uint16_t)0;
                    ha[c] = make_uint4(v[0] | (uint32_t)v[1] << 16, v[2] | (uint32_t)v[3] << 16,
                                       v[4] | (uint32_t)v[5] << 16, v[6] | (uint32_t)v[7] << 16);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < B_CH; ++c) {
            const int idx = tid + c * NT;
            if (B_TOT % NT != 0 && idx >= B_TOT) break;
            const int kp = idx % (kBK / 2), nc = (idx / (kBK / 2)) * BW;
            const int64_t gk = k0 + 2 * kp, gc = col0 + nc;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int64_t kk = gk + h;
                const bool fast = vec_ok && cols_full && kk < ke;
                if constexpr (MODE == 0) {
                    if (fast) {
                        const float4 v = *reinterpret_cast<const float4*>(Bf + kk * ldb + gc);
                        rb[c][h][0] = v.x; rb[c][h][1] = v.y; rb[c][h][2] = v.z; rb[c][h][3] = v.w;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            rb[c][h][e] = (kk < ke && gc + e < n) ? Bf[kk * ldb + gc + e] : 0.0f;
                    }
                } else {
                    if (fast) {
                        hb[c][h] = *reinterpret_cast<const uint4*>(Bh + kk * ldb + gc);
                    } else {
                        uint16_t v[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            v[e] = (kk < ke && gc + e < n) ? Bh[kk * ldb + gc + e] : (uint16_t)0;
                        hb[c][h] = make_uint4(v[0] | (uint32_t)v[1] << 16, v[2] | (uint32_t)v[3] << 16,
                                              v[4] | (uint32_t)v[5] << 16, v[6] | (uint32_t)v[7] << 16);
                    }
                }
            }
        }
    };

    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int c = 0; c < A_CH; ++c) {
            const int idx = tid + c * NT;
            if (A_TOT % NT != 0 && idx >= A_TOT) break;
            const int r = idx / (kBK / AW), kc = (idx % (kBK / AW)) * AW;
            if constexpr (MODE == 0) {
                uint32_t h[4], l[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) split2(ra[c][e], h[e], l[e]);
                *reinterpret_cast<uint2*>(&As[buf][0][r][kc]) = make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16);
                *reinterpret_cast<uint2*>(&As[buf][1][r][kc]) = make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16);
            } else {
                *reinterpret_cast<uint4*>(&As[buf][0][r][kc]) = ha[c];
            }
        }
#pragma unroll
        for (int c = 0; c < B_CH; ++c) {
            const int idx = tid + c * NT;
            if (B_TOT % NT != 0 && idx >= B_TOT) break;
            const int kp = idx % (kBK / 2), nc = (idx / (kBK / 2)) * BW;
            if constexpr (MODE == 0) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint32_t h0, l0, h1, l1;
                    split2(rb[c][0][e], h0, l0);
                    split2(rb[c][1][e], h1, l1);
                    *reinterpret_cast<uint32_t*>(&Bs[buf][0][nc + e][2 * kp]) = h0 | h1 << 16;
                    *reinterpret_cast<uint32_t*>(&Bs[buf][1][nc + e][2 * kp]) = l0 | l1 << 16;
                }
            } else {
                const uint32_t w0[4] = {hb[c][0].x, hb[c][0].y, hb[c][0].z, hb[c][0].w};
                const uint32_t w1[4] = {hb[c][1].x, hb[c][1].y, hb[c][1].z, hb[c][1].w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t lo16 = (w0[e / 2] >> (16 * (e % 2))) & 0xffffu;
                    const uint32_t hi16 = (w1[e / 2] >> (16 * (e % 2))) & 0xffffu;
                    *reinterpret_cast<uint32_t*>(&Bs[buf][0][nc + e][2 * kp]) = lo16 | hi16 << 16;
                }
            }
        }
    };

    const int64_t nkt = (ke - kb + kBK - 1) / kBK;
    if (nkt > 0) {
        load_tiles(kb);
        store_tiles(0);
        __syncthreads();
        for (int64_t kt = 0; kt < nkt; ++kt) {
            const int buf = (int)(kt & 1);
            if (kt + 1 < nkt) load_tiles(kb + (kt + 1) * kBK);
#pragma unroll
            for (int ks = 0; ks < kBK; ks += 16) {
                bf16x8 a[NP][FM], b[NP][FN];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        a[p][i] = *reinterpret_cast<const bf16x8*>(
                            &As[buf][p][wm * FM * 32 + i * 32 + lrow][ks + 8 * half]);
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        b[p][j] = *reinterpret_cast<const bf16x8*>(
                            &Bs[buf][p][wn * FN * 32 + j * 32 + lrow][ks + 8 * half]);
                }
                if constexpr (MODE == 0) {
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
            }
            if (kt + 1 < nkt) store_tiles(buf ^ 1);
            __syncthreads();
        }
    }

    const int r_sar = sigma & ((1 << sa.sar_levels) - 1);
    const int g_tar = sigma >> sa.sar_levels;
    const int per_group = (1 << sa.sar_levels) - 1;
    float* dst;
    int64_t ldd;
    if (r_sar == 0) {
        dst = C;
        ldd = ldc;
    } else {
        dst = temps + (int64_t)(g_tar * per_group + r_sar - 1) * sa.temp_stride;
        ldd = sa.ldt;
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int64_t gc = col0 + wn * FN * 32 + b * 32 + lrow;
            if (gc >= n) continue;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t gr = row0 + wm * FM * 32 + a * 32 + (i / 4) * 8 + half * 4 + (i % 4);
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

template <int BM, int BN, int WM, int WN, int MODE>
hipError_t launch_cfg(const Plan& p, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                      int64_t ldb, float* C, int64_t ldc, float* temps, const SliceArgs& sa_in, hipStream_t st) {
    const mm_plan_info& pi = p.info;
    SliceArgs sa = sa_in;
    sa.levels = pi.tar_levels + pi.sar_levels;
    sa.sar_levels = pi.sar_levels;
    sa.tk = kBK;
    sa.atomic_c = pi.tar_levels > 0;
    sa.temp_stride = p.temp_stride;
    sa.ldt = p.ldt;
    const int64_t tiles_m = ceil_div(m, BM), tiles_n = ceil_div(n, BN);
    const int64_t grid = tiles_m * tiles_n * pi.sched.split_k * sa.batch;
    if (grid == 0) return hipSuccess;
    const int64_t align_elems = MODE == 0 ? 4 : 8;
    const int vec_ok = (lda % align_elems == 0) && (ldb % align_elems == 0) && ((uintptr_t)A % 16 == 0) &&
                       ((uintptr_t)B % 16 == 0) && (sa.stride_a % align_elems == 0) &&
                       (sa.stride_b % align_elems == 0);
    ProfScope ps(MODE == 0 ? "bf16x3_tile" : "bf16_tile", st);
    hipLaunchKernelGGL((k_bf16_tile<BM, BN, WM, WN, MODE>), dim3((unsigned)grid), dim3(WM * WN * 64), 0, st, A, lda,
                       B, ldb, C, ldc, temps, m, n, k, tiles_m, tiles_n, sa, vec_ok);
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_mode(const Plan& p, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B,
                       int64_t ldb, float* C, int64_t ldc, float* temps, const SliceArgs& sa, hipStream_t st) {
    switch (p.info.sched.tile) {
        case 128: return launch_cfg<128, 128, 2, 2, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
        case 64: return launch_cfg<64, 64, 2, 2, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
        default: return launch_cfg<32, 32, 1, 1, MODE>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, sa, st);
    }
}

}  // namespace

hipError_t launch_bf16_tiles(const Plan& p, bool split3, int64_t m, int64_t n, int64_t k, const void* A, int64_t lda,
                             const void* B, int64_t ldb, float* C, int64_t ldc, float* temps, int64_t band_row0,
                             int64_t band_m, const SliceArgs& sa, hipStream_t st) {
    (void)m;
    const size_t esz = split3 ? 4 : 2;
    const void* Ab = static_cast<const char*>(A) + band_row0 * lda * esz;
    float* Cb = C + band_row0 * ldc;
    if (split3) return launch_mode<0>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    return launch_mode<1>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
}

}  // namespace starmm
