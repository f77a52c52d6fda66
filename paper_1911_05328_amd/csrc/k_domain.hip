// Domain check of integer-semiring operands (a debugging aid): the number of
// entries of a rows x cols int32 matrix outside [lo, hi].  One workgroup per
// row at a time, lanes along the row (coalesced), a wave reduction, then one
// atomic add per workgroup into the 64-bit device counter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.hpp"

namespace starmm {

namespace {

constexpr int kDomThreads = 256;

__global__ void __launch_bounds__(64) k_zero_u64(unsigned long long* __restrict__ p) {
    if (threadIdx.x == 0) *p = 0ull;
}

__global__ void __launch_bounds__(kDomThreads)
k_domain_count(const int32_t* __restrict__ X, int64_t ld, int64_t rows, int64_t cols, int32_t lo, int32_t hi,
               unsigned long long* __restrict__ count) {
    unsigned long long c = 0;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const int32_t* row = X + r * ld;
        for (int64_t q = threadIdx.x; q < cols; q += kDomThreads) {
            const int32_t v = row[q];
            c += (v < lo || v > hi) ? 1ull : 0ull;
        }
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    __shared__ unsigned long long part[kDomThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kDomThreads / 64; ++w) t += part[w];
        if (t) atomicAdd(count, t);
    }
}

}  // namespace

bool domain_bounds(mm_semiring_kind sr, int32_t flags, int32_t* lo, int32_t* hi) {
    const int32_t inf = 1 << 30;
    const bool wide = (flags & MM_FLAG_CHECKED_RANGE) != 0;
    switch (sr) {
        case MM_SR_MIN_PLUS: *lo = wide ? -inf : 0; *hi = inf; return true;
        case MM_SR_MAX_PLUS: *lo = -inf; *hi = wide ? inf - 1 : 0; return true;
        case MM_SR_MAX_MIN: *lo = INT32_MIN; *hi = INT32_MAX; return true;
        case MM_SR_OR_AND: *lo = 0; *hi = 1; return true;
        default: return false;
    }
}

hipError_t launch_domain_count(const int32_t* X, int64_t ld, int64_t rows, int64_t cols, int32_t lo, int32_t hi,
                               unsigned long long* count, bool zero_first, hipStream_t st) {
    if (zero_first) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, count);
    if (rows > 0 && cols > 0 && (lo != INT32_MIN || hi != INT32_MAX)) {
        const int64_t grid = std::min<int64_t>(rows, 8192);
        hipLaunchKernelGGL(k_domain_count, dim3((unsigned)grid), dim3(kDomThreads), 0, st, X, ld, rows, cols, lo, hi,
                           count);
    }
    return hipGetLastError();
}

}  // namespace starmm
