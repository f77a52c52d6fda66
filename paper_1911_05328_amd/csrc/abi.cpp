// C ABI entry points: argument validation (host, before any launch), planning
// and the launch sequence of each call.
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace starmm {

namespace {
thread_local std::string g_last_error;

mm_status hip_fail(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return MM_ERR_HIP;
}

bool ld_ok(int64_t ld, int64_t cols) { return ld >= (cols > 1 ? cols : 1); }

// STARMM_CHECK_DOMAIN set (to anything but "0"): integer-semiring calls count
// the entries of A, B and C outside the domain first, wait for the count and
// refuse the call if any; the counter is the caller's word when given,
// else one device word per device, allocated on first use and kept until
// the process ends.
bool check_domain_enabled() {
    const char* v = std::getenv("STARMM_CHECK_DOMAIN");
    return v && *v && std::strcmp(v, "0") != 0;
}

mm_status check_domain(mm_semiring_kind sr, int32_t flags, int64_t m, int64_t n, int64_t k, const void* A,
                       int64_t lda, const void* B, int64_t ldb, const void* C, int64_t ldc,
                       unsigned long long* counter, hipStream_t st) {
    int32_t lo, hi;
    if (!domain_bounds(sr, flags, &lo, &hi)) return MM_OK;
    static std::mutex mu;
    static unsigned long long* counters[64] = {};
    hipError_t e = hipSuccess;
    unsigned long long* cnt = counter;
    if (!cnt) {
        int dev = 0;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "domain check");
        if (dev < 0 || dev >= 64) return MM_OK;
        std::lock_guard<std::mutex> lock(mu);
        if (!counters[dev]) {
            e = hipMalloc(reinterpret_cast<void**>(&counters[dev]), sizeof(unsigned long long));
            if (e != hipSuccess) {
                counters[dev] = nullptr;
                return hip_fail(e, "domain check counter");
            }
        }
        cnt = counters[dev];
    }
    e = launch_domain_count((const int32_t*)A, lda, m, k, lo, hi, cnt, true, st);
    if (e == hipSuccess) e = launch_domain_count((const int32_t*)B, ldb, k, n, lo, hi, cnt, false, st);
    if (e == hipSuccess) e = launch_domain_count((const int32_t*)C, ldc, m, n, lo, hi, cnt, false, st);
    unsigned long long bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, cnt, sizeof bad, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "domain check");
    if (bad) {
        g_last_error = std::to_string(bad) + " entries of A, B, C outside [" + std::to_string(lo) + ", " +
                       std::to_string(hi) + "]";
        return MM_ERR_INVALID_ARG;
    }
    return MM_OK;
}

// Launch sequence of a planned (non-Strassen) product: for each band of C
// rows, the tile kernel over (tiles x slices), then the ordered merge of the
// band's temporaries.  Bands run one after another on the stream and reuse
// the same temporaries.
mm_status run_planned(const Plan& p, mm_semiring_kind sr, int64_t m, int64_t n, int64_t k, const void* A,
                      int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, void* ws,
                      hipStream_t st) {
    if (p.persistent) {
        const hipError_t e = launch_semiring_persistent(p, sr, m, n, k, (const int32_t*)A, lda, (const int32_t*)B,
                                                        ldb, (int32_t*)C, ldc, ws, st);
        return e == hipSuccess ? MM_OK : hip_fail(e, "mm_semiring persistent launch");
    }
    const int64_t band = p.band_rows;
    char* wsc = static_cast<char*>(ws);
    void* temps = wsc ? wsc + p.temps_off : nullptr;
    uint16_t* Ap = nullptr;
    uint16_t* Bp = nullptr;
    const bool one_plane = p.planes && (p.family == KF_BF16_MFMA || p.family == KF_F16_MFMA);
    if (one_plane) {
        // bf16 / fp16 inputs: one plane per operand, B transposed
        Ap = reinterpret_cast<uint16_t*>(wsc);
        Bp = Ap + plane_rows(m) * p.ldp;
        hipError_t e = launch_copy_rows16((const uint16_t*)A, lda, m, k, Ap, p.ldp, st);
        if (e == hipSuccess) e = launch_copy_transpose16((const uint16_t*)B, ldb, k, n, Bp, p.ldp, st);
        if (e != hipSuccess) return hip_fail(e, "mm_semiring planes");
    } else if (p.planes) {
        Ap = reinterpret_cast<uint16_t*>(wsc);
        Bp = Ap + 2 * plane_rows(m) * p.ldp;
        hipError_t e = launch_split_rows((const float*)A, lda, 0, m, k, Ap, p.ldp, 0, plane_rows(m) * p.ldp, 1, st);
        if (e == hipSuccess)
            e = launch_split_transpose((const float*)B, ldb, 0, k, n, Bp, p.ldp, 0, plane_rows(n) * p.ldp, 1, st);
        if (e != hipSuccess) return hip_fail(e, "mm_semiring split");
    }
    for (int64_t r0 = 0; r0 < m; r0 += band) {
        const int64_t bm = (m - r0) < band ? (m - r0) : band;
        hipError_t e = hipSuccess;
        switch (p.family) {
            case KF_SEMIRING_I32:
                e = launch_semiring_tiles(p, sr, m, n, k, (const int32_t*)A, lda, (const int32_t*)B, ldb,
                                          (int32_t*)C, ldc, (int32_t*)temps, r0, bm, st);
                if (e == hipSuccess)
                    e = launch_merge_i32(p, sr, (int32_t*)C, ldc, (const int32_t*)temps, r0, bm, n, st);
                break;
            case KF_F32_MFMA:
                e = launch_f32_tiles(p, m, n, k, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc,
                                     (float*)temps, r0, bm, SliceArgs(), st);
                if (e == hipSuccess) e = launch_merge_f32(p, (float*)C, ldc, (const float*)temps, r0, bm, n, st);
                break;
            case KF_BF16X3_MFMA:
            case KF_BF16_MFMA:
            case KF_F16_MFMA:
                if (one_plane) {
                    e = launch_bf16_tiles(p, p.family == KF_F16_MFMA ? 7 : 6, m, n, k, Ap, p.ldp, Bp, p.ldp,
                                          (float*)C, ldc, (float*)temps, r0, bm, SliceArgs(), st);
                } else if (p.planes) {
                    SliceArgs sa;
                    sa.a_plane = plane_rows(m) * p.ldp;
                    sa.b_plane = plane_rows(n) * p.ldp;
                    e = launch_bf16_tiles(p, 2, m, n, k, Ap, p.ldp, Bp, p.ldp, (float*)C, ldc, (float*)temps, r0, bm,
                                          sa, st);
                } else {
                    const int mode = p.family == KF_BF16X3_MFMA ? 0 : (p.family == KF_F16_MFMA ? 5 : 1);
                    e = launch_bf16_tiles(p, mode, m, n, k, A, lda, B, ldb, (float*)C, ldc, (float*)temps, r0, bm,
                                          SliceArgs(), st);
                }
                if (e == hipSuccess) e = launch_merge_f32(p, (float*)C, ldc, (const float*)temps, r0, bm, n, st);
                break;
            default:
                g_last_error = "kernel family not built";
                return MM_ERR_UNSUPPORTED;
        }
        if (e != hipSuccess) return hip_fail(e, "mm_semiring launch");
    }
    return MM_OK;
}

}  // namespace

bool semiring_args_ok(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B, int64_t ldb,
                      const void* C, int64_t ldc) {
    if (m < 0 || n < 0 || k < 0) return false;
    if (!ld_ok(lda, k) || !ld_ok(ldb, n) || !ld_ok(ldc, n)) return false;
    return !((m > 0 && k > 0 && !A) || (k > 0 && n > 0 && !B) || (m > 0 && n > 0 && !C));
}

mm_status semiring_call(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, const void* A,
                        int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, void* workspace,
                        size_t workspace_bytes, const mm_schedule* sched, bool use_selection,
                        unsigned long long* domain_counter, hipStream_t stream) {
    if (!semiring_args_ok(m, n, k, A, lda, B, ldb, C, ldc)) return MM_ERR_INVALID_ARG;
    if (!workspace_ok(workspace, workspace_bytes)) return MM_ERR_INVALID_ARG;
    mm_schedule chosen;
    if (!sched && use_selection && select_schedule(sr, dt, m, n, k, workspace_bytes, &chosen)) sched = &chosen;
    if (sched && (sched->strassen_depth > 0 || prec_fp16(sched->precision))) {
        Plan sp;
        mm_status st = make_plan(sr, dt, m, n, k, workspace_bytes, sched, &sp);
        if (st != MM_OK) return st;
        int32_t df = 0;
        while ((sp.info.sched.strassen_layout >> df) & 1) ++df;
        return star_strassen_run(m, n, k, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc,
                                 sched->star_depth, sched->strassen_depth, (mm_strassen_variant)sched->variant,
                                 (mm_precision)sched->precision, sched->tile, sp.info.sched.split_k, df, workspace,
                                 workspace_bytes, stream);
    }
    Plan p;
    mm_status st = make_plan(sr, dt, m, n, k, workspace_bytes, sched, &p);
    if (st != MM_OK) return st;
    if (m == 0 || n == 0 || k == 0) return MM_OK;
    if (p.family == KF_SEMIRING_I32 && check_domain_enabled()) {
        st = check_domain(sr, p.info.sched.flags, m, n, k, A, lda, B, ldb, C, ldc, domain_counter, stream);
        if (st != MM_OK) return st;
    }
    return run_planned(p, sr, m, n, k, A, lda, B, ldb, C, ldc, workspace, stream);
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

}  // namespace starmm

using namespace starmm;

extern "C" {

mm_status mm_plan(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, size_t workspace_bytes,
                  const mm_schedule* sched, mm_plan_info* out) {
    mm_schedule chosen;
    if (!sched && select_schedule(sr, dt, m, n, k, workspace_bytes, &chosen)) sched = &chosen;
    Plan p;
    mm_status st = make_plan(sr, dt, m, n, k, workspace_bytes, sched, &p);
    if (st == MM_OK && out) *out = p.info;
    return st;
}

size_t mm_workspace_bytes(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                          const mm_schedule* sched) {
    Plan p;
    if (make_plan(sr, dt, m, n, k, ~size_t(0) >> 1, sched, &p) != MM_OK) return 0;
    return (size_t)p.info.ws_bytes;
}

mm_status mm_semiring(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, const void* A,
                      int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, void* workspace,
                      size_t workspace_bytes, const mm_schedule* sched, void* stream) {
    return semiring_call(sr, dt, m, n, k, A, lda, B, ldb, C, ldc, workspace, workspace_bytes, sched, true, nullptr,
                         (hipStream_t)stream);
}

mm_status mm_domain_violations(mm_semiring_kind sr, int32_t flags, const int32_t* X, int64_t rows, int64_t cols,
                               int64_t ld, unsigned long long* count, void* stream) {
    int32_t lo, hi;
    if (!domain_bounds(sr, flags, &lo, &hi)) return MM_ERR_INVALID_ARG;
    if (flags & ~(MM_FLAG_NONDETERMINISTIC | MM_FLAG_SPLIT_IN_KERNEL | MM_FLAG_PERSISTENT | MM_FLAG_CHECKED_RANGE))
        return MM_ERR_INVALID_ARG;
    if (rows < 0 || cols < 0 || !ld_ok(ld, cols) || !count || (rows > 0 && cols > 0 && !X))
        return MM_ERR_INVALID_ARG;
    const hipError_t e = launch_domain_count(X, ld, rows, cols, lo, hi, count, true, (hipStream_t)stream);
    return e == hipSuccess ? MM_OK : hip_fail(e, "mm_domain_violations");
}

const char* mm_status_string(mm_status st) {
    switch (st) {
        case MM_OK: return "ok";
        case MM_ERR_INVALID_ARG: return "invalid argument";
        case MM_ERR_UNSUPPORTED: return "unsupported combination";
        case MM_ERR_WORKSPACE: return "workspace too small for the schedule";
        case MM_ERR_HIP: return "HIP runtime error";
        case MM_ERR_INCOMPLETE: return "a bounded wait of a persistent launch gave up: C is incomplete";
    }
    return "unknown status";
}

const char* mm_last_error(void) { return g_last_error.c_str(); }

mm_status mm_persistent_status(const void* workspace, size_t workspace_bytes, void* stream) {
    if (!workspace || (int64_t)workspace_bytes < persist_ctl_bytes(0)) return MM_ERR_INVALID_ARG;
    uint32_t err = 0;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&err, static_cast<const char*>(workspace) + kPersistErrorOffset, sizeof err,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "mm_persistent_status");
    if (err != 0) {
        g_last_error = "persistent launch: a slice waited past its bound for its slot group";
        return MM_ERR_INCOMPLETE;
    }
    return MM_OK;
}

int32_t mm_version(void) { return 100; }

mm_status mm_tile_order(int64_t tm, int64_t tn, int64_t* ti, int64_t* tj) {
    if (tm < 0 || tn < 0) return MM_ERR_INVALID_ARG;
    const int64_t tiles = tm * tn;
    if (tiles > (int64_t(1) << 26)) return MM_ERR_INVALID_ARG;
    if (tiles > 0 && (!ti || !tj)) return MM_ERR_INVALID_ARG;
    for (int64_t t = 0; t < tiles; ++t) recursion_tile(t, tm, tn, &ti[t], &tj[t]);
    return MM_OK;
}

}  // extern "C"
