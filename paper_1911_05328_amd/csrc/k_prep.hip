// Operand preparation for the pre-split bf16 product: fp32 operands become
// hi/lo bf16 planes (hi = bf16(x), lo = bf16(x - hi), both round to nearest
// even) in the k-tiled layout of tile_bf16.hpp, for both operands k-major,
// so the tile kernels stage them with plain (or direct-to-LDS) copies.
//   k_split_rows:      X (rows x cols) -> planes of X, rows x ldp.
//   k_split_transpose: X (rows x cols) -> planes of X^T, cols x ldp, through
//                      a 64 x 64 LDS tile (coalesced on both sides).
// A thread writes one 16-byte chunk (8 k values of one row) of each plane,
// threads in tiled order, so a wave writes 1 KB contiguous per plane.  Plane
// entries outside X (k in [cols, ldp), padding rows) are written as zeros.
// The fp16 form (F16) multiplies plane row r by scale[r] (an exact power of
// two, plane_rows long) before splitting; see k_pow2_scales below.
// 16-bit inputs (bf16 or fp16 operands of a one-plane product) are copied
// into one plane in the same layout by k_copy_rows16 / k_copy_transpose16.
// Both kernels take a batch index in blockIdx.y with element strides for
// the source and the planes (hi of product b at planes + b * plane_stride,
// lo at hi + lo_off).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {

constexpr int kT = 256;
constexpr int kRowT = 512;  // row-order copies and splits (faster than 256; the transposes are not)
constexpr int kTile = 64;

template <bool F16>
__global__ void __launch_bounds__(kRowT)
k_split_rows(const float* __restrict__ X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
             uint16_t* __restrict__ planes, int64_t ldp, int64_t plane_stride, int64_t lo_off, int64_t chunks,
             const float* __restrict__ scale) {
    const int64_t q = (int64_t)blockIdx.x * kRowT + threadIdx.x;
    if (q >= chunks) return;
    int64_t r, c0;
    chunk_coord(q, ldp, &r, &c0);
    X += (int64_t)blockIdx.y * x_stride;
    planes += (int64_t)blockIdx.y * plane_stride;
    const float sc = F16 ? scale[r] : 1.0f;
    const float* src = X + r * ldx + c0;
    float v[8];
    if (r < rows && c0 + 8 <= cols) {  // the 8 values through 16-byte loads
        const uint4 a = load16_any((gptr<const void>)src), b = load16_any((gptr<const void>)(src + 4));
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = __builtin_bit_cast(float, w[e]) * sc;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (r < rows && c0 + e < cols) ? src[e] * sc : 0.0f;
    }
    uint4 hi, lo;
    split_pack8<F16>(v, hi, lo);
    *reinterpret_cast<uint4*>(planes + q * 8) = hi;
    *reinterpret_cast<uint4*>(planes + lo_off + q * 8) = lo;
}

// One workgroup: X rows [r0, r0 + 64) x cols [c0, c0 + 64) -> plane rows
// (X columns) [c0, c0 + 64) x k (X rows) [r0, r0 + 64): 2 x 4 units.
template <bool F16>
__global__ void __launch_bounds__(kT)
k_split_transpose(const float* __restrict__ X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                  uint16_t* __restrict__ planes, int64_t ldp, int64_t plane_stride, int64_t lo_off,
                  int64_t prow_total, const float* __restrict__ scale) {
    __shared__ float t[kTile][kTile + 1];
    const int64_t tiles_c = (prow_total + kTile - 1) / kTile;
    const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * kTile, c0 = (int64_t)(blockIdx.x % tiles_c) * kTile;
    X += (int64_t)blockIdx.y * x_stride;
    planes += (int64_t)blockIdx.y * plane_stride;
    if (r0 + kTile <= rows && c0 + kTile <= cols) {
        // whole tile inside X: 16-byte loads (16 threads per 256-byte tile row)
        const int cx = (threadIdx.x & 15) * 4, ry = threadIdx.x >> 4;  // 16 x 16
#pragma unroll
        for (int i = ry; i < kTile; i += kT / 16) {
            const uint4 v = load16_any((gptr<const void>)(X + (r0 + i) * ldx + c0 + cx));
            t[i][cx] = __builtin_bit_cast(float, v.x), t[i][cx + 1] = __builtin_bit_cast(float, v.y);
            t[i][cx + 2] = __builtin_bit_cast(float, v.z), t[i][cx + 3] = __builtin_bit_cast(float, v.w);
        }
    } else {
        const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 64 x 4
        for (int i = ty; i < kTile; i += kT / kTile) {
            const int64_t r = r0 + i, c = c0 + tx;
            t[i][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.0f;
        }
    }
    __syncthreads();
    // 8 units of 64 chunks; thread w handles chunk w % 64 of units w / 64, w / 64 + 4
    for (int w = threadIdx.x; w < 8 * 64; w += kT) {
        const int u = w >> 6, p = w & 63;
        const int ub = u >> 2, uk = u & 3;  // unit row block (of 2), k block (of 4)
        const int ri = p >> 1, c = (p & 1) ^ tiled_swz(ri);
        const int64_t prow = c0 + ub * kPlaneRowBlock + ri;          // plane row = X column
        const int64_t k0 = r0 + uk * kPlaneKBlock + c * 8;            // plane k = X row
        if (prow >= prow_total || k0 >= ldp) continue;
        const float sc = F16 ? scale[prow] : 1.0f;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[uk * kPlaneKBlock + c * 8 + e][ub * kPlaneRowBlock + ri] * sc;
        uint4 hi, lo;
        split_pack8<F16>(v, hi, lo);
        const int64_t off = tiled_off(prow, k0, ldp);
        *reinterpret_cast<uint4*>(planes + off) = hi;
        *reinterpret_cast<uint4*>(planes + lo_off + off) = lo;
    }
}

// One plane of 16-bit values X (rows x cols) in the k-tiled layout: a thread
// writes one 16-byte chunk (8 k of one row); zeros outside X.
__global__ void __launch_bounds__(kRowT)
k_copy_rows16(const uint16_t* __restrict__ X, int64_t ldx, int64_t rows, int64_t cols, uint16_t* __restrict__ plane,
              int64_t ldp, int64_t chunks) {
    const int64_t q = (int64_t)blockIdx.x * kRowT + threadIdx.x;
    if (q >= chunks) return;
    int64_t r, c0;
    chunk_coord(q, ldp, &r, &c0);
    const uint16_t* src = X + r * ldx + c0;
    if (r < rows && c0 + 8 <= cols) {  // the 8 values through 16-byte loads
        *reinterpret_cast<uint4*>(plane + q * 8) = load16_any((gptr<const void>)src);
        return;
    }
    uint32_t v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (r < rows && c0 + e < cols) ? src[e] : 0u;
    *reinterpret_cast<uint4*>(plane + q * 8) =
        make_uint4(v[0] | v[1] << 16, v[2] | v[3] << 16, v[4] | v[5] << 16, v[6] | v[7] << 16);
}

// 16-bit X (rows x cols) -> one plane of X^T (cols plane rows x ldp), through
// a 64 x 64 LDS tile as in k_split_transpose.
__global__ void __launch_bounds__(kT)
k_copy_transpose16(const uint16_t* __restrict__ X, int64_t ldx, int64_t rows, int64_t cols,
                   uint16_t* __restrict__ plane, int64_t ldp, int64_t prow_total) {
    __shared__ uint16_t t[kTile][kTile + 2];
    const int64_t tiles_c = (prow_total + kTile - 1) / kTile;
    const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * kTile, c0 = (int64_t)(blockIdx.x % tiles_c) * kTile;
    if (r0 + kTile <= rows && c0 + kTile <= cols) {
        // whole tile inside X: 16-byte loads (8 threads per 128-byte tile
        // row), stored into LDS as four 4-byte words
        const int cx = (threadIdx.x & 7) * 8, ry = threadIdx.x >> 3;  // 8 x 32
#pragma unroll
        for (int i = ry; i < kTile; i += kT / 8) {
            const uint4 v = load16_any((gptr<const void>)(X + (r0 + i) * ldx + c0 + cx));
            uint32_t* d = reinterpret_cast<uint32_t*>(&t[i][cx]);
            d[0] = v.x, d[1] = v.y, d[2] = v.z, d[3] = v.w;
        }
    } else {
        const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 64 x 4
        for (int i = ty; i < kTile; i += kT / kTile) {
            const int64_t r = r0 + i, c = c0 + tx;
            t[i][tx] = (r < rows && c < cols) ? X[r * ldx + c] : (uint16_t)0;
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < 8 * 64; w += kT) {
        const int u = w >> 6, p = w & 63;
        const int ub = u >> 2, uk = u & 3;
        const int ri = p >> 1, c = (p & 1) ^ tiled_swz(ri);
        const int64_t prow = c0 + ub * kPlaneRowBlock + ri;
        const int64_t k0 = r0 + uk * kPlaneKBlock + c * 8;
        if (prow >= prow_total || k0 >= ldp) continue;
        uint32_t v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[uk * kPlaneKBlock + c * 8 + e][ub * kPlaneRowBlock + ri];
        *reinterpret_cast<uint4*>(plane + tiled_off(prow, k0, ldp)) =
            make_uint4(v[0] | v[1] << 16, v[2] | v[3] << 16, v[4] | v[5] << 16, v[6] | v[7] << 16);
    }
}

// ---- scales of the fp16 split
//
// fp16 keeps 11 significant bits only between 2^-14 and 65504, so before the
// split every row of A (column of B) is multiplied by a power of two chosen
// from its largest |entry|.  Strassen leaf row x mixes source rows off[I] + x
// of the 2^d row blocks, so its scale comes from the largest of those rows'
// maxima, times a bound on how much the pre-additions can grow an entry.

// out[r] = max_c |X[r, c]|: one wave per row.  VEC: 16-byte loads (X and
// ldx 4-aligned, cols % 4 == 0), four in flight per lane.
__device__ inline float absmax4(float4 v) { return fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))); }

template <bool VEC>
__global__ void __launch_bounds__(kT)
k_absmax_rows(const float* __restrict__ X, int64_t ldx, int64_t rows, int64_t cols, float* __restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (r >= rows) return;
    const int lane = threadIdx.x & 63;
    float mx = 0.0f;
    if constexpr (VEC) {
        const float4* row = reinterpret_cast<const float4*>(X + r * ldx);
        const int64_t c4 = cols / 4;
        int64_t c = lane;
        for (; c + 192 < c4; c += 256) {
            const float4 a = row[c], b = row[c + 64], d = row[c + 128], e = row[c + 192];
            mx = fmaxf(mx, fmaxf(fmaxf(absmax4(a), absmax4(b)), fmaxf(absmax4(d), absmax4(e))));
        }
        for (; c < c4; c += 64) mx = fmaxf(mx, absmax4(row[c]));
    } else {
        for (int64_t c = lane; c < cols; c += 64) mx = fmaxf(mx, fabsf(X[r * ldx + c]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) out[r] = mx;
}

__global__ void __launch_bounds__(kT) k_zero_f32(float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) out[i] = 0.0f;
}

// out[c] = max_r |X[r, c]| (out zeroed first): a thread folds rows_per rows
// of CW consecutive columns (CW = 4: 16-byte loads, X and ldx 4-aligned,
// cols % 4 == 0), then an atomic max on each float's bits (non-negative
// floats order like their bit patterns).
template <int CW>
__global__ void __launch_bounds__(kT)
k_absmax_cols(const float* __restrict__ X, int64_t ldx, int64_t rows, int64_t cols, int64_t rows_per,
              float* __restrict__ out) {
    const int64_t c = ((int64_t)blockIdx.x * kT + threadIdx.x) * CW;
    if (c >= cols) return;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
    float mx[CW];
#pragma unroll
    for (int j = 0; j < CW; ++j) mx[j] = 0.0f;
    if constexpr (CW == 4) {
        int64_t r = r0;
        for (; r + 4 <= r1; r += 4) {
            float4 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const float4*>(X + (r + q) * ldx + c);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                mx[0] = fmaxf(mx[0], fabsf(v[q].x));
                mx[1] = fmaxf(mx[1], fabsf(v[q].y));
                mx[2] = fmaxf(mx[2], fabsf(v[q].z));
                mx[3] = fmaxf(mx[3], fabsf(v[q].w));
            }
        }
        for (; r < r1; ++r) {
            const float4 v = *reinterpret_cast<const float4*>(X + r * ldx + c);
            mx[0] = fmaxf(mx[0], fabsf(v.x));
            mx[1] = fmaxf(mx[1], fabsf(v.y));
            mx[2] = fmaxf(mx[2], fabsf(v.z));
            mx[3] = fmaxf(mx[3], fabsf(v.w));
        }
    } else {
        for (int64_t r = r0; r < r1; ++r) mx[0] = fmaxf(mx[0], fabsf(X[r * ldx + c]));
    }
#pragma unroll
    for (int j = 0; j < CW; ++j) atomicMax(reinterpret_cast<unsigned int*>(out) + c + j, __float_as_uint(mx[j]));
}

// Leaf row x (of leaf_rows; rows up to prow get scale 1):
//   bound = growth * max_{I: x < ext[I]} absmax[off[I] + x]
//   scale = 2^(13 - ilogb(bound)), so bound * scale < 2^14; 1 if bound is 0.
__global__ void __launch_bounds__(kT)
k_pow2_scales(const float* __restrict__ absmax, PathTable paths, int nblk, float growth, int64_t leaf_rows,
              int64_t prow, float* __restrict__ scale, float* __restrict__ unscale) {
    const int64_t x = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (x >= prow) return;
    float mx = 0.0f;
    if (x < leaf_rows)
        for (int I = 0; I < nblk; ++I)
            if (x < paths.ext[I]) mx = fmaxf(mx, absmax[paths.off[I] + x]);
    const float bound = growth * mx;
    int e = 0;
    if (bound > 0.0f && bound <= 3.0e38f) {
        e = 13 - ilogbf(bound);
        e = e < -120 ? -120 : (e > 120 ? 120 : e);
    }
    scale[x] = ldexpf(1.0f, e);
    unscale[x] = ldexpf(1.0f, -e);
}

}  // namespace

hipError_t launch_split_rows(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                             uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off, int64_t batch,
                             hipStream_t st, const float* f16_scale) {
    if (rows == 0 || ldp == 0 || batch == 0) return hipSuccess;
    if (ldp % kPlaneKBlock != 0) return hipErrorInvalidValue;
    ProfScope ps("split_rows", st);
    const int64_t chunks = plane_rows(rows) * ldp / 8;
    const dim3 grid((unsigned)ceil_div(chunks, kRowT), (unsigned)batch);
    if (f16_scale)
        hipLaunchKernelGGL(k_split_rows<true>, grid, dim3(kRowT), 0, st, X, ldx, x_stride, rows, cols, planes, ldp,
                           plane_stride, lo_off, chunks, f16_scale);
    else
        hipLaunchKernelGGL(k_split_rows<false>, grid, dim3(kRowT), 0, st, X, ldx, x_stride, rows, cols, planes, ldp,
                           plane_stride, lo_off, chunks, f16_scale);
    return hipGetLastError();
}

hipError_t launch_split_transpose(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                                  uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off,
                                  int64_t batch, hipStream_t st, const float* f16_scale) {
    if (cols == 0 || ldp == 0 || batch == 0) return hipSuccess;
    if (ldp % kPlaneKBlock != 0) return hipErrorInvalidValue;
    ProfScope ps("split_transpose", st);
    // tiles cover every plane row (padding rows included) and every k < ldp
    const int64_t prow_total = plane_rows(cols);
    const dim3 grid((unsigned)(ceil_div(ldp, kTile) * ceil_div(prow_total, kTile)), (unsigned)batch);
    if (f16_scale)
        hipLaunchKernelGGL(k_split_transpose<true>, grid, dim3(kT), 0, st, X, ldx, x_stride, rows, cols, planes, ldp,
                           plane_stride, lo_off, prow_total, f16_scale);
    else
        hipLaunchKernelGGL(k_split_transpose<false>, grid, dim3(kT), 0, st, X, ldx, x_stride, rows, cols, planes,
                           ldp, plane_stride, lo_off, prow_total, f16_scale);
    return hipGetLastError();
}

hipError_t launch_copy_rows16(const uint16_t* X, int64_t ldx, int64_t rows, int64_t cols, uint16_t* plane,
                              int64_t ldp, hipStream_t st) {
    if (rows == 0 || ldp == 0) return hipSuccess;
    if (ldp % kPlaneKBlock != 0) return hipErrorInvalidValue;
    ProfScope ps("split_rows", st);
    const int64_t chunks = plane_rows(rows) * ldp / 8;
    hipLaunchKernelGGL(k_copy_rows16, dim3((unsigned)ceil_div(chunks, kRowT)), dim3(kRowT), 0, st, X, ldx, rows, cols,
                       plane, ldp, chunks);
    return hipGetLastError();
}

hipError_t launch_copy_transpose16(const uint16_t* X, int64_t ldx, int64_t rows, int64_t cols, uint16_t* plane,
                                   int64_t ldp, hipStream_t st) {
    if (cols == 0 || ldp == 0) return hipSuccess;
    if (ldp % kPlaneKBlock != 0) return hipErrorInvalidValue;
    ProfScope ps("split_transpose", st);
    const int64_t prow_total = plane_rows(cols);
    hipLaunchKernelGGL(k_copy_transpose16, dim3((unsigned)(ceil_div(ldp, kTile) * ceil_div(prow_total, kTile))),
                       dim3(kT), 0, st, X, ldx, rows, cols, plane, ldp, prow_total);
    return hipGetLastError();
}

hipError_t launch_absmax_rows(const float* X, int64_t ldx, int64_t rows, int64_t cols, float* out, hipStream_t st) {
    if (rows == 0) return hipSuccess;
    ProfScope ps("f16_scales", st);
    const dim3 grid((unsigned)ceil_div(rows, kT / 64));
    if (((uintptr_t)X & 15) == 0 && ldx % 4 == 0 && cols % 4 == 0)
        hipLaunchKernelGGL(k_absmax_rows<true>, grid, dim3(kT), 0, st, X, ldx, rows, cols, out);
    else
        hipLaunchKernelGGL(k_absmax_rows<false>, grid, dim3(kT), 0, st, X, ldx, rows, cols, out);
    return hipGetLastError();
}

hipError_t launch_absmax_cols(const float* X, int64_t ldx, int64_t rows, int64_t cols, float* out, hipStream_t st) {
    if (cols == 0) return hipSuccess;
    ProfScope ps("f16_scales", st);
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)ceil_div(cols, kT)), dim3(kT), 0, st, out, cols);
    if (rows == 0) return hipGetLastError();
    const bool vec = ((uintptr_t)X & 15) == 0 && ldx % 4 == 0 && cols % 4 == 0;
    const int cw = vec ? 4 : 1;
    const int64_t col_blocks = ceil_div(cols, (int64_t)kT * cw);
    // about 2048 workgroups, each thread folding at least 64 rows; at most
    // 65535 row chunks
    const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(ceil_div(rows, 64), ceil_div(2048, col_blocks)));
    const int64_t rows_per = std::max<int64_t>(ceil_div(rows, chunks), ceil_div(rows, 65535));
    const dim3 grid((unsigned)col_blocks, (unsigned)ceil_div(rows, rows_per));
    if (vec)
        hipLaunchKernelGGL(k_absmax_cols<4>, grid, dim3(kT), 0, st, X, ldx, rows, cols, rows_per, out);
    else
        hipLaunchKernelGGL(k_absmax_cols<1>, grid, dim3(kT), 0, st, X, ldx, rows, cols, rows_per, out);
    return hipGetLastError();
}

hipError_t launch_pow2_scales(const float* absmax, const PathTable& paths, int depth, float growth,
                              int64_t leaf_rows, float* scale, float* unscale, hipStream_t st) {
    const int64_t prow = plane_rows(leaf_rows);
    if (prow == 0) return hipSuccess;
    ProfScope ps("f16_scales", st);
    hipLaunchKernelGGL(k_pow2_scales, dim3((unsigned)ceil_div(prow, kT)), dim3(kT), 0, st, absmax, paths,
                       1 << depth, growth, leaf_rows, prow, scale, unscale);
    return hipGetLastError();
}

}  // namespace starmm
