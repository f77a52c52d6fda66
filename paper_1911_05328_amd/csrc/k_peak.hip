// Microbenchmarks of the resources the kernels are bounded by, so achieved
// rates can be reported against what this chip sustains as well as against
// its datasheet: int32 add/min3 VALU throughput, bf16 and fp32 MFMA
// throughput (register operands only), and a streaming HBM copy.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace starmm {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWG = 256;

// 16 independent (min,+) accumulators; one loop step is 16 x (2 adds + 1 min3)
// = 48 VALU ops per lane.
__global__ void __launch_bounds__(kWG) k_peak_valu(int64_t iters, uint32_t* out) {
    uint32_t acc[16], b[16];
    const uint32_t t = threadIdx.x + blockIdx.x * 7u;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        acc[j] = 0x3fffffffu - t - j;
        b[j] = t * 3u + j;
    }
    uint32_t a0 = t & 1023u, a1 = (t >> 3) & 1023u;
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t s0 = a0 + b[j], s1 = a1 + b[j];
            acc[j] = acc[j] < s0 ? acc[j] : s0;
            acc[j] = acc[j] < s1 ? acc[j] : s1;
        }
        a0 += 1u;
        a1 += 3u;
    }
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) r ^= acc[j];
    if (r == 0x12345678u) out[blockIdx.x] = r;  // keeps the loop live
}

// 4 independent 32x32x16 bf16 MFMA chains per wave.
__global__ void __launch_bounds__(kWG) k_peak_mfma_bf16(int64_t iters, float* out) {
    f32x16 c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i) c[q][i] = 0.0f;
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = (__bf16)(float)((threadIdx.x + i) & 7);
        b[i] = (__bf16)(float)((threadIdx.x * 3 + i) & 7);
    }
    for (int64_t it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[q], 0, 0, 0);
    float r = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) r += c[q][threadIdx.x & 15];
    if (r == -1.0f) out[blockIdx.x] = r;
}

// 4 independent 32x32x2 fp32 MFMA chains per wave.
__global__ void __launch_bounds__(kWG) k_peak_mfma_f32(int64_t iters, float* out) {
    f32x16 c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i) c[q][i] = 0.0f;
    const float a = (float)(threadIdx.x & 7), b = (float)((threadIdx.x * 3) & 7);
    for (int64_t it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c[q], 0, 0, 0);
    float r = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) r += c[q][threadIdx.x & 15];
    if (r == -1.0f) out[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kWG) k_peak_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kWG) dst[i] = src[i];
}

}  // namespace

}  // namespace starmm

using namespace starmm;

extern "C" mm_status mm_microbench(int32_t kind, int64_t iters, void* buf_a, void* buf_b, int64_t bytes, double* work,
                                   void* stream) {
    if (!work || iters < 0) return MM_ERR_INVALID_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return MM_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    const int grid = cus * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    switch (kind) {
        case 0:  // int32 VALU lane-ops
            if (!buf_a) return MM_ERR_INVALID_ARG;
            hipLaunchKernelGGL(k_peak_valu, dim3(grid), dim3(kWG), 0, st, iters, (uint32_t*)buf_a);
            *work = (double)grid * kWG * iters * 48.0;
            break;
        case 1:  // bf16 MFMA flops
            if (!buf_a) return MM_ERR_INVALID_ARG;
            hipLaunchKernelGGL(k_peak_mfma_bf16, dim3(grid), dim3(kWG), 0, st, iters, (float*)buf_a);
            *work = (double)grid * (kWG / 64) * iters * 4.0 * (2.0 * 32 * 32 * 16);
            break;
        case 2:  // fp32 MFMA flops
            if (!buf_a) return MM_ERR_INVALID_ARG;
            hipLaunchKernelGGL(k_peak_mfma_f32, dim3(grid), dim3(kWG), 0, st, iters, (float*)buf_a);
            *work = (double)grid * (kWG / 64) * iters * 4.0 * (2.0 * 32 * 32 * 2);
            break;
        case 3: {  // HBM bytes moved (read + write)
            if (!buf_a || !buf_b || bytes < 16) return MM_ERR_INVALID_ARG;
            const int64_t n16 = bytes / 16;
            hipLaunchKernelGGL(k_peak_copy, dim3(cus * 16), dim3(kWG), 0, st, (const uint4*)buf_a, (uint4*)buf_b, n16);
            *work = 2.0 * n16 * 16;
            break;
        }
        default:
            return MM_ERR_INVALID_ARG;
    }
    return hipGetLastError() == hipSuccess ? MM_OK : MM_ERR_HIP;
}
