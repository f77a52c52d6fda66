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
// Both kernels take a batch index in blockIdx.y with element strides for
// the source and the planes (hi of product b at planes + b * plane_stride,
// lo at hi + lo_off).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {

constexpr int kT = 256;
constexpr int kTile = 64;

__global__ void __launch_bounds__(kT)
k_split_rows(const float* __restrict__ X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
             uint16_t* __restrict__ planes, int64_t ldp, int64_t plane_stride, int64_t lo_off, int64_t chunks) {
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (q >= chunks) return;
    int64_t r, c0;
    chunk_coord(q, ldp, &r, &c0);
    X += (int64_t)blockIdx.y * x_stride;
    planes += (int64_t)blockIdx.y * plane_stride;
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (r < rows && c0 + e < cols) ? X[r * ldx + c0 + e] : 0.0f;
    uint4 hi, lo;
    split_pack8(v, hi, lo);
    *reinterpret_cast<uint4*>(planes + q * 8) = hi;
    *reinterpret_cast<uint4*>(planes + lo_off + q * 8) = lo;
}

// One workgroup: X rows [r0, r0 + 64) x cols [c0, c0 + 64) -> plane rows
// (X columns) [c0, c0 + 64) x k (X rows) [r0, r0 + 64): 2 x 4 units.
__global__ void __launch_bounds__(kT)
k_split_transpose(const float* __restrict__ X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                  uint16_t* __restrict__ planes, int64_t ldp, int64_t plane_stride, int64_t lo_off,
                  int64_t prow_total) {
    __shared__ float t[kTile][kTile + 1];
    const int64_t tiles_c = (prow_total + kTile - 1) / kTile;
    const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * kTile, c0 = (int64_t)(blockIdx.x % tiles_c) * kTile;
    X += (int64_t)blockIdx.y * x_stride;
    planes += (int64_t)blockIdx.y * plane_stride;
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 64 x 4
    for (int i = ty; i < kTile; i += kT / kTile) {
        const int64_t r = r0 + i, c = c0 + tx;
        t[i][tx] = (r < rows && c < cols) ? X[r * ldx + c] : 0.0f;
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
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = t[uk * kPlaneKBlock + c * 8 + e][ub * kPlaneRowBlock + ri];
        uint4 hi, lo;
        split_pack8(v, hi, lo);
        const int64_t off = tiled_off(prow, k0, ldp);
        *reinterpret_cast<uint4*>(planes + off) = hi;
        *reinterpret_cast<uint4*>(planes + lo_off + off) = lo;
    }
}

}  // namespace

hipError_t launch_split_rows(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                             uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off, int64_t batch,
                             hipStream_t st) {
    if (rows == 0 || ldp == 0 || batch == 0) return hipSuccess;
    if (ldp % kPlaneKBlock != 0) return hipErrorInvalidValue;
    ProfScope ps("split_rows", st);
    const int64_t chunks = plane_rows(rows) * ldp / 8;
    hipLaunchKernelGGL(k_split_rows, dim3((unsigned)ceil_div(chunks, kT), (unsigned)batch), dim3(kT), 0, st, X, ldx,
                       x_stride, rows, cols, planes, ldp, plane_stride, lo_off, chunks);
    return hipGetLastError();
}

hipError_t launch_split_transpose(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                                  uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off,
                                  int64_t batch, hipStream_t st) {
    if (cols == 0 || ldp == 0 || batch == 0) return hipSuccess;
    if (ldp % kPlaneKBlock != 0) return hipErrorInvalidValue;
    ProfScope ps("split_transpose", st);
    // tiles cover every plane row (padding rows included) and every k < ldp
    const int64_t prow_total = plane_rows(cols);
    const int64_t grid = ceil_div(ldp, kTile) * ceil_div(prow_total, kTile);
    hipLaunchKernelGGL(k_split_transpose, dim3((unsigned)grid, (unsigned)batch), dim3(kT), 0, st, X, ldx, x_stride,
                       rows, cols, planes, ldp, plane_stride, lo_off, prow_total);
    return hipGetLastError();
}

}  // namespace starmm
