// fp32 (+,x) base-case tiles on MFMA (v_mfma_f32_32x32x2_f32): the plain
// 8-way recursion flattened into output tiles (eq. mm-dac; Fig. mm-n2 is the
// split_k = 1 schedule), with the same k-slice / temporary / merge scheme as
// the semiring kernel.
//
// MFMA lane layout (32x32x2, fp32): lane l supplies A[row l%32][k slot l/32]
// and B[k slot l/32][col l%32]; accumulator register i of lane l holds
// C[row 8*(i/4) + 4*(l/32) + i%4][col l%32].  Within a group of 8 k values,
// lane half h takes k = 4h + j in the j-th MFMA (j = 0..3), so one 16-byte
// LDS read feeds four MFMAs; A and B use the same k assignment, so the sum
// over the group is unchanged.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "kcommon.hpp"

namespace starmm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBK = 16;
constexpr int kApad = 4;  // As row stride BK + 4 floats: conflict-free 16-byte reads
constexpr int kBpad = 8;  // Bs row stride BN + 8 floats: the two lane halves hit disjoint banks

template <int BM, int BN, int WM, int WN>
__global__ void __launch_bounds__(WM * WN * 64)
k_f32_tile(const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb,
           float* __restrict__ C, int64_t ldc, float* __restrict__ temps, int64_t m, int64_t n, int64_t k,
           int64_t tiles_m, int64_t tiles_n, SliceArgs sa, int vec_ok) {
    constexpr int NT = WM * WN * 64;
    constexpr int FM = BM / WM / 32, FN = BN / WN / 32;  // 32x32 blocks per wave
    constexpr int A_CHUNKS = BM * kBK / 4 / NT;
    constexpr int B_CHUNKS = BN * kBK / 4 / NT;
    static_assert(FM >= 1 && FN >= 1 && A_CHUNKS >= 1 && B_CHUNKS >= 1, "bad tile");

    __shared__ __attribute__((aligned(16))) float As[2][BM][kBK + kApad];
    __shared__ __attribute__((aligned(16))) float Bs[2][kBK][BN + kBpad];

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
    A += bidx * sa.stride_a;
    B += bidx * sa.stride_b;
    C += bidx * sa.stride_c;
    const int64_t row0 = ti * BM, col0 = tj * BN;
    int64_t kb, ke;
    slice_k_range(sigma, sa.levels, k, sa.tk, &kb, &ke);

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

    const bool rows_full = row0 + BM <= m;
    const bool cols_full = col0 + BN <= n;
    float4 ra[A_CHUNKS], rb[B_CHUNKS];

    auto load_tiles = [&](int64_t k0) {
        const bool k_full = k0 + kBK <= ke;
#pragma unroll
        for (int c = 0; c < A_CHUNKS; ++c) {
            const int idx = tid + c * NT;
            const int r = idx / (kBK / 4), kc = (idx % (kBK / 4)) * 4;
            const int64_t gr = row0 + r, gk = k0 + kc;
            if (vec_ok && k_full && (rows_full || gr < m)) {
                ra[c] = *reinterpret_cast<const float4*>(A + gr * lda + gk);
            } else {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (gr < m && gk + e < ke) ? A[gr * lda + gk + e] : 0.0f;
                ra[c] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
#pragma unroll
        for (int c = 0; c < B_CHUNKS; ++c) {
            const int idx = tid + c * NT;
            const int r = idx / (BN / 4), nc = (idx % (BN / 4)) * 4;
            const int64_t gk = k0 + r, gc = col0 + nc;
            if (vec_ok && cols_full && gk < ke) {
                rb[c] = *reinterpret_cast<const float4*>(B + gk * ldb + gc);
            } else {
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (gk < ke && gc + e < n) ? B[gk * ldb + gc + e] : 0.0f;
                rb[c] = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int c = 0; c < A_CHUNKS; ++c) {
            const int idx = tid + c * NT;
            const int r = idx / (kBK / 4), kc = (idx % (kBK / 4)) * 4;
            *reinterpret_cast<float4*>(&As[buf][r][kc]) = ra[c];
        }
#pragma unroll
        for (int c = 0; c < B_CHUNKS; ++c) {
            const int idx = tid + c * NT;
            const int r = idx / (BN / 4), nc = (idx % (BN / 4)) * 4;
            *reinterpret_cast<float4*>(&Bs[buf][r][nc]) = rb[c];
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
            for (int kk = 0; kk < kBK; kk += 8) {
                float4 av[FM];
                float bv[FN][4];
#pragma unroll
                for (int a = 0; a < FM; ++a)
                    av[a] = *reinterpret_cast<const float4*>(&As[buf][wm * FM * 32 + a * 32 + lrow][kk + 4 * half]);
#pragma unroll
                for (int b = 0; b < FN; ++b)
#pragma unroll
                    for (int j = 0; j < 4; ++j) bv[b][j] = Bs[buf][kk + 4 * half + j][wn * FN * 32 + b * 32 + lrow];
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int a = 0; a < FM; ++a)
#pragma unroll
                        for (int b = 0; b < FN; ++b) {
                            const float x = j == 0 ? av[a].x : j == 1 ? av[a].y : j == 2 ? av[a].z : av[a].w;
                            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(x, bv[b][j], acc[a][b], 0, 0, 0);
                        }
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
        dst = temps + bidx * sa.temp_batch_stride + (int64_t)(g_tar * per_group + r_sar - 1) * sa.temp_stride;
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

// Ordered merge of float temporaries (recursion order: neighbours first).
template <int NS>
__global__ void __launch_bounds__(256)
k_merge_f32(float* __restrict__ C, int64_t ldc, const float* __restrict__ temps, int64_t m, int64_t n, int groups,
            int atomic_c, int64_t temp_stride, int64_t ldt, int64_t c_batch_stride, int64_t temp_batch_stride) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * n) return;
    C += (int64_t)blockIdx.y * c_batch_stride;
    temps += (int64_t)blockIdx.y * temp_batch_stride;
    const int64_t i = idx / n, j = idx % n;
    for (int g = 0; g < groups; ++g) {
        float v[NS];
        v[0] = atomic_c ? 0.0f : C[i * ldc + j];
#pragma unroll
        for (int r = 1; r < NS; ++r) v[r] = temps[(int64_t)(g * (NS - 1) + r - 1) * temp_stride + i * ldt + j];
#pragma unroll
        for (int w = 1; w < NS; w *= 2)
#pragma unroll
            for (int q = 0; q + w < NS; q += 2 * w) v[q] = v[q] + v[q + w];
        if (atomic_c)
            atomicAdd(&C[i * ldc + j], v[0]);
        else
            C[i * ldc + j] = v[0];
    }
}

template <int BM, int BN, int WM, int WN>
hipError_t launch_cfg(const Plan& p, int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B,
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
    const int vec_ok = (lda % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) &&
                       (sa.stride_a % 4 == 0) && (sa.stride_b % 4 == 0);
    ProfScope ps("f32_tile", st);
    hipLaunchKernelGGL((k_f32_tile<BM, BN, WM, WN>), dim3((unsigned)grid), dim3(WM * WN * 64), 0, st, A, lda, B, ldb,
                       C, ldc, temps, m, n, k, tiles_m, tiles_n, sa, vec_ok);
    return hipGetLastError();
}

template <int NS>
hipError_t merge_ns(const Plan& p, float* C, int64_t ldc, const float* temps, int64_t m, int64_t n, int64_t batch,
                    int64_t c_bs, int64_t t_bs, hipStream_t st) {
    const int64_t total = m * n;
    if (total == 0 || batch == 0) return hipSuccess;
    ProfScope ps("merge", st);
    hipLaunchKernelGGL((k_merge_f32<NS>), dim3((unsigned)ceil_div(total, 256), (unsigned)batch), dim3(256), 0, st, C,
                       ldc, temps, m, n, 1 << p.info.tar_levels, (int)(p.info.tar_levels > 0), p.temp_stride, p.ldt,
                       c_bs, t_bs);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_f32_tiles(const Plan& p, int64_t m, int64_t n, int64_t k, const float* A, int64_t lda,
                            const float* B, int64_t ldb, float* C, int64_t ldc, float* temps, int64_t band_row0,
                            int64_t band_m, const SliceArgs& sa, hipStream_t st) {
    (void)m;
    const float* Ab = A + band_row0 * lda;
    float* Cb = C + band_row0 * ldc;
    switch (p.info.sched.tile) {
        case 128: return launch_cfg<128, 128, 2, 2>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
        case 64: return launch_cfg<64, 64, 2, 2>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
        default: return launch_cfg<32, 32, 1, 1>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, sa, st);
    }
}

hipError_t launch_merge_f32(const Plan& p, float* C, int64_t ldc, const float* temps, int64_t band_row0,
                            int64_t band_m, int64_t n, hipStream_t st, int64_t batch, int64_t c_batch_stride,
                            int64_t temp_batch_stride) {
    float* Cb = C + band_row0 * ldc;
    const int64_t b = batch, cs = c_batch_stride, ts = temp_batch_stride;
    switch (p.info.sar_levels) {
        case 0: return hipSuccess;
        case 1: return merge_ns<2>(p, Cb, ldc, temps, band_m, n, b, cs, ts, st);
        case 2: return merge_ns<4>(p, Cb, ldc, temps, band_m, n, b, cs, ts, st);
        case 3: return merge_ns<8>(p, Cb, ldc, temps, band_m, n, b, cs, ts, st);
        case 4: return merge_ns<16>(p, Cb, ldc, temps, band_m, n, b, cs, ts, st);
        case 5: return merge_ns<32>(p, Cb, ldc, temps, band_m, n, b, cs, ts, st);
        default: return merge_ns<64>(p, Cb, ldc, temps, band_m, n, b, cs, ts, st);
    }
}

}  // namespace starmm
