// Strassen path (Sec. strassen): placeholder until the kernels land.
#include "internal.hpp"

extern "C" {

size_t mm_strassen_workspace_bytes(int64_t, int64_t, int64_t, int32_t, mm_strassen_variant, mm_precision) {
    return 0;
}

mm_status mm_strassen(int64_t, int64_t, int64_t, const float*, int64_t, const float*, int64_t, float*, int64_t,
                      int32_t, mm_strassen_variant, mm_precision, void*, size_t, void*) {
    return MM_ERR_UNSUPPORTED;
}

}
