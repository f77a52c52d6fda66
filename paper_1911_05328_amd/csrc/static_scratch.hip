// mm_semiring_static: mm_semiring for callers that cannot allocate device
// memory.  The workspace is a file-scope device array of fixed size (one
// copy per GPU, held until the process ends); its device address is looked
// up once per device with hipGetSymbolAddress and only that address is ever
// handed to kernels or copies.  Every call on one GPU shares the array.
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace starmm {

namespace {

// Bytes ahead of the workspace part: the debugging mode's domain counter.
constexpr size_t kCounterBytes = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kCounterBytes + MM_STATIC_SCRATCH_BYTES];

std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on
// that device); nullptr with the last error set on failure.
unsigned char* device_scratch() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_last_error(std::string("mm_semiring_static: hipGetDevice: ") + hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_last_error("mm_semiring_static: device ordinal " + std::to_string(dev) + " beyond the supported " +
                       std::to_string(kMaxDevices));
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_last_error(std::string("mm_semiring_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch[dev] = static_cast<unsigned char*>(ptr);
    }
    return g_scratch[dev];
}

}  // namespace

}  // namespace starmm

using namespace starmm;

extern "C" {

mm_status mm_semiring_static(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, const void* A,
                             int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc,
                             const mm_schedule* sched, void* stream) {
    // everything is checked on the host before the first HIP call
    if (!semiring_args_ok(m, n, k, A, lda, B, ldb, C, ldc)) return MM_ERR_INVALID_ARG;
    if (sched && (sched->flags & MM_FLAG_PERSISTENT)) {
        set_last_error("mm_semiring_static: MM_FLAG_PERSISTENT needs a caller workspace (its status word)");
        return MM_ERR_UNSUPPORTED;
    }
    {
        // the schedule (explicit or the planner's) must fit the array
        Plan p;
        const mm_status st = make_plan(sr, dt, m, n, k, MM_STATIC_SCRATCH_BYTES, sched, &p);
        if (st == MM_ERR_WORKSPACE && sched) {
            Plan unbounded;
            const int64_t need = make_plan(sr, dt, m, n, k, ~size_t(0) >> 1, sched, &unbounded) == MM_OK
                                     ? unbounded.info.ws_bytes
                                     : -1;
            set_last_error("mm_semiring_static: the schedule needs " +
                           (need >= 0 ? std::to_string(need) : std::string("more")) +
                           " bytes of scratch, the static scratch holds " +
                           std::to_string((long long)MM_STATIC_SCRATCH_BYTES));
        }
        if (st != MM_OK) return st;
    }
    if (m == 0 || n == 0 || k == 0) return MM_OK;
    unsigned char* s = device_scratch();
    if (!s) return MM_ERR_HIP;
    return semiring_call(sr, dt, m, n, k, A, lda, B, ldb, C, ldc, s + kCounterBytes, MM_STATIC_SCRATCH_BYTES,
                         sched, false, reinterpret_cast<unsigned long long*>(s), (hipStream_t)stream);
}

}  // extern "C"
