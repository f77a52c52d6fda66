// Operand preparation for the pre-split bf16 product: fp32 operands become
// hi/lo bf16 planes (hi = bf16(x), lo = bf16(x - hi), both round to nearest
// even), laid out k-contiguous for both operands, so the tile kernel stages
// them with plain 16-byte copies.
//   k_split_rows:      X (rows x cols) -> planes of X, rows x ldp.
//   k_split_transpose: X (rows x cols) -> planes of X^T, cols x ldp, through
//                      a 64 x 64 LDS tile (coalesced on both sides).
// Columns [cols, ldp) of a plane row are written as zeros.  Both kernels
// take a batch index in blockIdx.y with element strides for the source and
// the planes (hi of product b at planes + b * plane_stride, lo at
// hi + lo_off).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {

constexpr int kT = 256;
constexpr int kTile = 64;

__device__ inline void split_pack8(const float* x, uint4& hi, uint4& lo) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) split2(x[e], h[e], l[e]);
    hi = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16);
    lo = make_uint4(l[0] | l[1] << 16, l[2] | l[3] << 16, l[4] | l[5] << 16, l[6] | l[7] << 16);
}

__global__ void __launch_bounds__(kT)
k_split_rows(const float* __restrict__ X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
             uint16_t* __restrict__ planes, int64_t ldp, int64_t plane_stride, int64_t lo_off) {
    const int64_t chunks = ldp / 8;
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= rows * chunks) return;
    const int64_t r = idx / chunks, c0 = (idx % chunks) * 8;
    X += (int64_t)blockIdx.y * x_stride;
    planes += (int64_t)blockIdx.y * plane_stride;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = c0 + e < cols ? X[r * ldx + c0 + e] : 0.0f;
    uint4 hi, lo;
    split_pack8(v, hi, lo);
    *reinterpret_cast<uint4*>(planes + r * ldp + c0) = hi;
    *reinterpret_cast<uint4*>(planes + lo_off + r * ldp + c0) = lo;
}

__global__ void __launch_bounds__(kT)
k_split_transpose(const float* __restrict__ X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                  uint16_t* __restrict__ planes, int64_t ldp, int64_t plane_stride, int64_t lo_off) {
    __shared__ float t[kTile][kTile + 1];
    const int64_t tiles_c = (cols + kTile - 1) / kTile;
    const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * kTile, c0 = (int64_t)(blockIdx.x % tiles_c) * kTile;
    X += (int64_t)blockIdx.y * x_stride;
    planes += (int64_t)blockIdx.y * plane_stride;
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 64 x 4
    for (int i = ty; i < kTile; i += kT / kTile) {
        const int64_t r = r0 + i, c = c0 + tx;
        t[i][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.0f;
    }
    __syncthreads();
    // output row c (a column of X), 8 consecutive entries r0 + 8q .. +7
    for (int w = threadIdx.x; w < kTile * (kTile / 8); w += kT) {
        const int cc = w / (kTile / 8), q = w % (kTile / 8);
        const int64_t c = c0 + cc, r = r0 + 8 * q;
        if (c >= cols || r >= ldp) continue;
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[8 * q + e][cc];
        uint4 hi, lo;
        split_pack8(v, hi, lo);
        *reinterpret_cast<uint4*>(planes + c * ldp + r) = hi;
        *reinterpret_cast<uint4*>(planes + lo_off + c * ldp + r) = lo;
    }
}

}  // namespace

hipError_t launch_split_rows(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                             uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off, int64_t batch,
                             hipStream_t st) {
    if (rows == 0 || ldp == 0 || batch == 0) return hipSuccess;
    ProfScope ps("split_rows", st);
    hipLaunchKernelGGL(k_split_rows, dim3((unsigned)ceil_div(rows * (ldp / 8), kT), (unsigned)batch), dim3(kT), 0,
                       st, X, ldx, x_stride, rows, cols, planes, ldp, plane_stride, lo_off);
    return hipGetLastError();
}

hipError_t launch_split_transpose(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                                  uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off,
                                  int64_t batch, hipStream_t st) {
    if (cols == 0 || ldp == 0 || batch == 0) return hipSuccess;
    ProfScope ps("split_transpose", st);
    // tiles must also cover the zero columns [rows, ldp) of every plane row
    const int64_t grid = ceil_div(ldp, kTile) * ceil_div(cols, kTile);
    hipLaunchKernelGGL(k_split_transpose, dim3((unsigned)grid, (unsigned)batch), dim3(kT), 0, st, X, ldx, x_stride,
                       rows, cols, planes, ldp, plane_stride, lo_off);
    return hipGetLastError();
}

}  // namespace starmm
