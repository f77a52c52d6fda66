// One level of a general bilinear scheme (the bilinear circuit of the
// closing remarks of Sec. strassen, eq. bilinear) around the batched
// base-product tiles: the pre-addition forms every product's operands
// straight into k-tiled bf16 hi/lo planes, the post-addition combines the
// products into the blocks of C.  Coefficients arrive as kernel arguments.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bilinear.hpp"
#include "internal.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// workgroup sizes (measured: 512 threads made the post-addition and the
// pre-addition of 2 x 2 grids faster than 256, the 4 x 4 pre-addition slower)
template <int G>
constexpr int kPreT = G <= 2 ? 512 : 256;
constexpr int kPostT = 512;

// Pre-addition of one side.  A thread owns 8 consecutive tiled positions of
// the leaf planes (8 consecutive k of one leaf row), reads that run from
// every block of its operand's grid, and for each product r writes
// sum_p coef[r][p] X_p (fp32, ascending p) as bf16 hi/lo chunks of leaf r.
// SIDE_B: X = B (k x n) read in place, the leaves being B^T operands: leaf
// row x is column x of block-column s, k position y is row y of block-row l,
// coefficient index l*G + s.  Otherwise X = A: leaf row x of block-row s,
// k position y of block-column l, coefficient index s*G + l.  Positions
// outside the operand (padding rows, k past its end) read as 0.
template <int G, bool SIDE_B>
__global__ void __launch_bounds__(kPreT<G>)
k_bilinear_pre(const float* __restrict__ X, int64_t ldx, BlockTable rows, BlockTable ks,
               uint16_t* __restrict__ out, int64_t prow, int64_t ldo, int64_t leaf_stride, int64_t lo_off,
               BilinearSide cf) {
    int64_t pos = ((int64_t)blockIdx.x * kPreT<G> + threadIdx.x) * 8;
    if (pos >= prow * ldo) return;
    const int64_t ku = ldo / kPlaneKBlock;
    if constexpr (SIDE_B) {
        // units in k-block-major order: consecutive workgroups take the
        // row blocks (32 columns of B each) of one k-block, so B is read
        // along its rows rather than down 16-row strips
        const int64_t lin = pos >> 9, nrb = prow / kPlaneRowBlock;
        pos = ((lin % nrb) * ku + lin / nrb) * 512 + (pos & 511);
    }
    const int64_t unit = pos >> 9;
    const int p = (int)(pos & 511), ri = p >> 4, c = ((p >> 3) & 1) ^ tiled_swz(ri);
    const int64_t x = (unit / ku) * kPlaneRowBlock + ri;
    const int64_t y0 = (unit % ku) * kPlaneKBlock + c * 8;
    float v[G * G][8];
#pragma unroll
    for (int q = 0; q < G * G; ++q) {
        const int s = SIDE_B ? q % G : q / G, l = SIDE_B ? q / G : q % G;
        const bool row_ok = x < rows.ext[s];
        if constexpr (!SIDE_B) {
            const float* src = X + (rows.off[s] + x) * ldx + ks.off[l] + y0;
            if (row_ok && y0 + 8 <= ks.ext[l] && ((uintptr_t)src & 15) == 0) {
                const float4 a = reinterpret_cast<const float4*>(src)[0];
                const float4 b = reinterpret_cast<const float4*>(src)[1];
                v[q][0] = a.x, v[q][1] = a.y, v[q][2] = a.z, v[q][3] = a.w;
                v[q][4] = b.x, v[q][5] = b.y, v[q][6] = b.z, v[q][7] = b.w;
                continue;
            }
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t y = y0 + e;
            const bool ok = row_ok && y < ks.ext[l];
            const int64_t idx = SIDE_B ? (ks.off[l] + y) * ldx + rows.off[s] + x : (rows.off[s] + x) * ldx + ks.off[l] + y;
            v[q][e] = ok ? X[idx] : 0.0f;
        }
    }
    for (int r = 0; r < cf.products; ++r) {
        float sum[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int q = 0; q < G * G; ++q) {
            const int co = cf.coef[r * G * G + q];
            if (co == 0) continue;
            const float f = (float)co;
#pragma unroll
            for (int e = 0; e < 8; ++e) sum[e] += f * v[q][e];
        }
        uint32_t h[8], lo[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            h[e] = bf16_bits(sum[e]);
            lo[e] = bf16_bits(sum[e] - bf16_value(h[e]));
        }
        uint16_t* dst = out + r * leaf_stride + pos;
        *reinterpret_cast<uint4*>(dst) = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16,
                                                    h[6] | h[7] << 16);
        *reinterpret_cast<uint4*>(dst + lo_off) = make_uint4(lo[0] | lo[1] << 16, lo[2] | lo[3] << 16,
                                                             lo[4] | lo[5] << 16, lo[6] | lo[7] << 16);
    }
}

// Post-addition: a thread per NV consecutive leaf positions (x, y0 ..
// y0 + NV - 1); C block c gains sum_r gamma[c][r] P_r(x, y) (fp32, ascending
// r) where the block holds that position.  NV = 4: 16-byte product loads
// (rows padded to a multiple of 4, 16-byte aligned) and 16-byte C updates
// where a block's columns and C's alignment allow.
template <int G, int NV>
__global__ void __launch_bounds__(kPostT)
k_bilinear_post(const float* __restrict__ P, int64_t ldp, int64_t leaf_stride, BlockTable rows, BlockTable cols,
                float* __restrict__ C, int64_t ldc, int64_t leaf_rows, int64_t leaf_cols, BilinearOut cf) {
    const int64_t groups = (leaf_cols + NV - 1) / NV;
    const int64_t col_blocks = (groups + kPostT - 1) / kPostT;
    const int64_t x = (int64_t)blockIdx.x / col_blocks;
    const int64_t y0 = (((int64_t)blockIdx.x % col_blocks) * kPostT + threadIdx.x) * NV;
    if (y0 >= leaf_cols || x >= leaf_rows) return;
    float acc[G * G][NV];
#pragma unroll
    for (int q = 0; q < G * G; ++q)
#pragma unroll
        for (int e = 0; e < NV; ++e) acc[q][e] = 0.0f;
    // eight products' values loaded at once (the loads overlap), then
    // combined in ascending r
    constexpr int kChunk = 8;
    const float* src = P + x * ldp + y0;
    for (int r0 = 0; r0 < cf.products; r0 += kChunk) {
        float pr[kChunk][NV];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            if constexpr (NV == 4) {  // (products are read once: non-temporal loads)
                const f32x4 v = r0 + u < cf.products
                                    ? __builtin_nontemporal_load(
                                          reinterpret_cast<const f32x4*>(src + (r0 + u) * leaf_stride))
                                    : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                pr[u][0] = v.x, pr[u][1] = v.y, pr[u][2] = v.z, pr[u][3] = v.w;
            } else {
                pr[u][0] = r0 + u < cf.products ? src[(r0 + u) * leaf_stride] : 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            const int r = r0 + u;
            if (r >= cf.products) break;
#pragma unroll
            for (int q = 0; q < G * G; ++q) {
                const int co = cf.coef[q * cf.products + r];
                if (co != 0) {
#pragma unroll
                    for (int e = 0; e < NV; ++e) acc[q][e] += (float)co * pr[u][e];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < G * G; ++q) {
        const int i = q / G, j = q % G;
        if (x >= rows.ext[i]) continue;
        float* c = C + (rows.off[i] + x) * ldc + cols.off[j] + y0;
        const int64_t ye = cols.ext[j] - y0;  // columns e < ye exist
        if constexpr (NV == 4) {
            if (ye >= 4 && ((uintptr_t)c & 15) == 0) {
                float4 v = *reinterpret_cast<float4*>(c);
                v.x += acc[q][0], v.y += acc[q][1], v.z += acc[q][2], v.w += acc[q][3];
                *reinterpret_cast<float4*>(c) = v;
                continue;
            }
        }
#pragma unroll
        for (int e = 0; e < NV; ++e)
            if (e < ye) c[e] += acc[q][e];
    }
}

template <int G>
hipError_t pre_g(bool side_b, const float* X, int64_t ldx, const BlockTable& rows, const BlockTable& ks,
                 uint16_t* out, int64_t prow, int64_t ldo, int64_t leaf_stride, int64_t lo_off, const BilinearSide& cf,
                 hipStream_t st) {
    const dim3 grid((unsigned)ceil_div(prow * ldo / 8, kPreT<G>));
    if (side_b)
        hipLaunchKernelGGL((k_bilinear_pre<G, true>), grid, dim3(kPreT<G>), 0, st, X, ldx, rows, ks, out, prow, ldo,
                           leaf_stride, lo_off, cf);
    else
        hipLaunchKernelGGL((k_bilinear_pre<G, false>), grid, dim3(kPreT<G>), 0, st, X, ldx, rows, ks, out, prow, ldo,
                           leaf_stride, lo_off, cf);
    return hipGetLastError();
}

template <int G>
hipError_t post_g(const float* P, int64_t ldp, int64_t leaf_stride, const BlockTable& rows, const BlockTable& cols,
                  float* C, int64_t ldc, int64_t lr, int64_t lc, const BilinearOut& cf, hipStream_t st) {
    // 16-byte product loads stay inside each padded row
    if (ldp % 4 == 0 && leaf_stride % 4 == 0 && ldp >= round_up(lc, 4) && ((uintptr_t)P & 15) == 0) {
        const dim3 grid((unsigned)(lr * ceil_div(ceil_div(lc, 4), kPostT)));
        hipLaunchKernelGGL((k_bilinear_post<G, 4>), grid, dim3(kPostT), 0, st, P, ldp, leaf_stride, rows, cols, C,
                           ldc, lr, lc, cf);
    } else {
        const dim3 grid((unsigned)(lr * ceil_div(lc, kPostT)));
        hipLaunchKernelGGL((k_bilinear_post<G, 1>), grid, dim3(kPostT), 0, st, P, ldp, leaf_stride, rows, cols, C,
                           ldc, lr, lc, cf);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bilinear_pre(int g, bool side_b, const float* X, int64_t ldx, const BlockTable& rows,
                               const BlockTable& ks, uint16_t* out, int64_t prow, int64_t ldo, int64_t leaf_stride,
                               int64_t lo_off, const BilinearSide& cf, hipStream_t st) {
    if (prow == 0 || ldo == 0) return hipSuccess;
    if (ldo % kPlaneKBlock != 0 || prow % kPlaneRowBlock != 0) return hipErrorInvalidValue;
    if ((uint64_t)ceil_div(prow * ldo / 8, 256) > UINT32_MAX) return hipErrorInvalidValue;  // (the smaller size)
    ProfScope ps("bilinear_pre", st);
    switch (g) {
        case 1: return pre_g<1>(side_b, X, ldx, rows, ks, out, prow, ldo, leaf_stride, lo_off, cf, st);
        case 2: return pre_g<2>(side_b, X, ldx, rows, ks, out, prow, ldo, leaf_stride, lo_off, cf, st);
        case 3: return pre_g<3>(side_b, X, ldx, rows, ks, out, prow, ldo, leaf_stride, lo_off, cf, st);
        case 4: return pre_g<4>(side_b, X, ldx, rows, ks, out, prow, ldo, leaf_stride, lo_off, cf, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bilinear_post(int g, const float* P, int64_t ldp, int64_t leaf_stride, const BlockTable& rows,
                                const BlockTable& cols, float* C, int64_t ldc, int64_t lr, int64_t lc,
                                const BilinearOut& cf, hipStream_t st) {
    if (lr == 0 || lc == 0) return hipSuccess;
    if ((uint64_t)(lr * ceil_div(lc, kPostT)) > UINT32_MAX) return hipErrorInvalidValue;
    ProfScope ps("bilinear_post", st);
    switch (g) {
        case 1: return post_g<1>(P, ldp, leaf_stride, rows, cols, C, ldc, lr, lc, cf, st);
        case 2: return post_g<2>(P, ldp, leaf_stride, rows, cols, C, ldc, lr, lc, cf, st);
        case 3: return post_g<3>(P, ldp, leaf_stride, rows, cols, C, ldc, lr, lc, cf, st);
        case 4: return post_g<4>(P, ldp, leaf_stride, rows, cols, C, ldc, lr, lc, cf, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace starmm
