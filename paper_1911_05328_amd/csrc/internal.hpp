// Internal declarations shared by the host planner, the ABI layer and the
// kernel launchers.  Not part of the public interface (include/starmm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "kcommon.hpp"
#include "starmm.h"
#include "strassen_tables.hpp"

namespace starmm {

constexpr int64_t kInf = int64_t(1) << 30;  // sentinel infinity of (min,+) / (max,+)
constexpr int kMaxSplit = 64;               // largest k-split (2^6 slices)
constexpr int kMaxStrassenDepth = 3;
constexpr int kMaxStarStrassen = 3;  // 8-way levels above Strassen levels
constexpr size_t kAlign = 256;              // workspace sub-buffer alignment
constexpr int kBf16BKHost = 32;             // k per staged tile of the bf16 kernels

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
// A caller's workspace: none, or a non-null pointer aligned to kAlign (the
// sub-buffers are laid out at kAlign offsets from it and read with 16-byte
// and direct-to-LDS loads).
inline bool workspace_ok(const void* ws, size_t bytes) {
    return bytes == 0 || (ws && (reinterpret_cast<uintptr_t>(ws) % kAlign) == 0);
}
// Rows of a k-tiled bf16 plane holding r rows (whole 32-row units).
inline int64_t plane_rows(int64_t r) { return round_up(r, 32); }
// Row length of a k-tiled plane for k values: whole 32-deep k-tiles
// (slice boundaries), zero-padded.
inline int64_t plane_ld(int64_t k) { return round_up(k > 1 ? k : 1, kBf16BKHost); }
inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
inline int ilog2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

// Element size of C for a dtype (BF16 inputs accumulate into float C).
inline size_t c_elem_size(mm_dtype) { return 4; }
inline size_t ab_elem_size(mm_dtype dt) { return dt == MM_DT_BF16 || dt == MM_DT_F16 ? 2 : 4; }

inline bool prec_fp16(int p) { return p == MM_PREC_FP16X3 || p == MM_PREC_FP16X3_HIACC; }
inline bool prec_hiacc(int p) { return p == MM_PREC_BF16X3_HIACC || p == MM_PREC_FP16X3_HIACC; }

// Which kernel family serves a (semiring, dtype, precision) triple.
enum KernelFamily {
    KF_SEMIRING_I32 = 0,  // VALU (min,+)/(max,+)
    KF_F32_MFMA = 1,      // fp32 MFMA
    KF_BF16X3_MFMA = 2,   // split fp32 -> bf16 hi/lo, 3 products
    KF_BF16_MFMA = 3,     // bf16 inputs
    KF_F16_MFMA = 4       // fp16 inputs
};

struct Plan {
    mm_plan_info info;
    KernelFamily family;
    int64_t band_rows;  // rows of C per pass (multiple of tile, or m)
    int64_t ldt;        // leading dimension of a temporary
    int64_t temp_stride;  // elements between consecutive temporaries
    bool planes;          // operands through k-tiled planes in the workspace (BF16x3: hi/lo; bf16 / fp16
                          // inputs: one plane each)
    bool fp16 = false;    // FP16x3: the planes hold fp16 hi/lo of row/column-scaled operands
    int64_t ldp;          // plane row length: k rounded up to a whole staged tile, zero-filled
    int64_t planes_bytes; // bytes of the A and B^T planes at the start of the workspace
    int64_t temps_off;    // byte offset of the temporaries in the workspace
    bool persistent;      // integer semirings: one persistent launch, ring of slot groups
    int64_t groups;       // slot groups of the ring (split_k slots each); 0 when split_k = 1
};

// Persistent integer-semiring launch: workspace = control block (item
// counter, error word, per-group owner tile and arrival count) then
// groups x split_k slots of tile x tile int32.
inline int64_t persist_ctl_bytes(int64_t groups) { return round_up(16 + 12 * groups, kAlign); }
constexpr int64_t kPersistErrorOffset = 8;  // byte offset of the control block's error word
inline int64_t persist_groups(int64_t split_k) { return split_k > 1 ? ceil_div(MM_PERSIST_SLOTS, split_k) : 0; }

// Fill `plan` for a mm_semiring call.  Pure host code; returns the status
// the call would return before launching anything.
mm_status make_plan(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                    size_t workspace_bytes, const mm_schedule* sched, Plan* plan);

// The schedule a call without one takes from the loaded timings or cost
// model (false: none loaded or none applies; the built-in planner decides).
bool select_schedule(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, size_t budget,
                     mm_schedule* out);

void set_last_error(const std::string& msg);

// mm_semiring's argument check: sizes, leading dimensions, null pointers
// where entries exist.
bool semiring_args_ok(int64_t m, int64_t n, int64_t k, const void* A, int64_t lda, const void* B, int64_t ldb,
                      const void* C, int64_t ldc);

// mm_semiring's validation, planning and launches.  use_selection: a call
// without a schedule may take the loaded timings / cost model; otherwise the
// built-in planner decides.  domain_counter: one device word the
// STARMM_CHECK_DOMAIN debugging mode counts into (nullptr: a word the
// library allocates once per device).
mm_status semiring_call(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, const void* A,
                        int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, void* workspace,
                        size_t workspace_bytes, const mm_schedule* sched, bool use_selection,
                        unsigned long long* domain_counter, hipStream_t stream);

// Brackets one kernel launch with HIP events on its stream when profiling
// is enabled (mm_profile_enable); a no-op otherwise.
class ProfScope {
public:
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

private:
    const char* name_;
    hipStream_t st_;
    void* a_;
};

// ---- kernel launchers (each returns hipSuccess or the launch error) ----

// Semiring tile kernel over one band of C rows.
//  mode 0: C = C (+) acc, mode 1: atomic (+) into C, mode 2: temp <- acc
// (the mode is derived per slice from the plan inside the kernel).
hipError_t launch_semiring_tiles(const Plan& p, mm_semiring_kind sr, int64_t m, int64_t n, int64_t k,
                                 const int32_t* A, int64_t lda, const int32_t* B, int64_t ldb,
                                 int32_t* C, int64_t ldc, int32_t* temps, int64_t band_row0,
                                 int64_t band_m, hipStream_t st);

// Persistent integer-semiring product (MM_FLAG_PERSISTENT): init kernel
// for the control block, then one persistent launch over all (tile, slice)
// items; ws is the plan's workspace.
hipError_t launch_semiring_persistent(const Plan& p, mm_semiring_kind sr, int64_t m, int64_t n, int64_t k,
                                      const int32_t* A, int64_t lda, const int32_t* B, int64_t ldb, int32_t* C,
                                      int64_t ldc, void* ws, hipStream_t st);

// Ordered merge of a band's temporaries into C: for every TAR group, the
// SAR slices are reduced in recursion (binary tree) order and (+)-ed into C.
// The documented input domain [lo, hi] of an integer semiring under the
// schedule flags (false for (+,x)); the number of entries of X outside it
// into *count (device), after zeroing it when zero_first.
bool domain_bounds(mm_semiring_kind sr, int32_t flags, int32_t* lo, int32_t* hi);
hipError_t launch_domain_count(const int32_t* X, int64_t ld, int64_t rows, int64_t cols, int32_t lo, int32_t hi,
                               unsigned long long* count, bool zero_first, hipStream_t st);

hipError_t launch_merge_i32(const Plan& p, mm_semiring_kind sr, int32_t* C, int64_t ldc,
                            const int32_t* temps, int64_t band_row0, int64_t band_m, int64_t n,
                            hipStream_t st);
hipError_t launch_merge_f32(const Plan& p, float* C, int64_t ldc, const float* temps,
                            int64_t band_row0, int64_t band_m, int64_t n, hipStream_t st,
                            int64_t batch = 1, int64_t c_batch_stride = 0, int64_t temp_batch_stride = 0);

// fp32 MFMA tiles (plain recursion flattened), same slice/temporary scheme.
// `sa` carries the batch / overwrite fields; the slice fields come from p.
hipError_t launch_f32_tiles(const Plan& p, int64_t m, int64_t n, int64_t k, const float* A,
                            int64_t lda, const float* B, int64_t ldb, float* C, int64_t ldc,
                            float* temps, int64_t band_row0, int64_t band_m, const SliceArgs& sa,
                            hipStream_t st);

// bf16 MFMA tiles.  mode 0: fp32 operands split into hi/lo in the kernel
// (three products); 1: bf16 operands (one product); 2: pre-split planes
// (A hi/lo m x k, B^T hi/lo n x k; lo offsets in sa.a_plane / sa.b_plane);
// 4: as 2 with fp16 planes; 5: fp16 operands (one fp16 product); 6 / 7: one
// bf16 / fp16 plane per operand (A, B^T), one product, 256 or 128 tiles only.
hipError_t launch_bf16_tiles(const Plan& p, int mode, int64_t m, int64_t n, int64_t k,
                             const void* A, int64_t lda, const void* B, int64_t ldb, float* C,
                             int64_t ldc, float* temps, int64_t band_row0, int64_t band_m,
                             const SliceArgs& sa, hipStream_t st);

// Split fp32 operands into bf16 hi/lo planes (k_prep.hip); see there.
hipError_t launch_split_rows(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                             uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off, int64_t batch,
                             hipStream_t st, const float* f16_scale = nullptr);
// X (rows x cols) -> planes of X^T (cols plane rows); f16_scale: fp16 planes
// with plane row r (= column r of X) multiplied by f16_scale[r].
hipError_t launch_split_transpose(const float* X, int64_t ldx, int64_t x_stride, int64_t rows, int64_t cols,
                                  uint16_t* planes, int64_t ldp, int64_t plane_stride, int64_t lo_off,
                                  int64_t batch, hipStream_t st, const float* f16_scale = nullptr);
// 16-bit operands (bf16 / fp16) copied into one k-tiled plane: X itself
// (rows plane rows) or X^T (cols plane rows); zeros outside X.
hipError_t launch_copy_rows16(const uint16_t* X, int64_t ldx, int64_t rows, int64_t cols, uint16_t* plane,
                              int64_t ldp, hipStream_t st);
hipError_t launch_copy_transpose16(const uint16_t* X, int64_t ldx, int64_t rows, int64_t cols, uint16_t* plane,
                                   int64_t ldp, hipStream_t st);
// Scales of the fp16 split: out[r] = max_c |X[r, c]|, out[c] = max_r |X[r, c]|,
// and per leaf row x the power of two 2^(13 - ilogb(growth * max over the
// source rows paths.off[I] + x)) with its inverse (plane_rows(leaf_rows)
// entries each; padding rows get 1).
hipError_t launch_absmax_rows(const float* X, int64_t ldx, int64_t rows, int64_t cols, float* out, hipStream_t st);
hipError_t launch_absmax_cols(const float* X, int64_t ldx, int64_t rows, int64_t cols, float* out, hipStream_t st);
hipError_t launch_pow2_scales(const float* absmax, const PathTable& paths, int depth, float growth,
                              int64_t leaf_rows, float* scale, float* unscale, hipStream_t st);

// Strassen pre-additions of one operand (side 0 = A with alpha, 1 = B with
// beta) into 7^depth leaf operands, and post-additions of 7^depth products
// into C (C <- C + result).  f64: additions in double.
// fix: the depth-first round (kAllFree: every level breadth-first, all 7^depth
// leaves); only the leaves under the fixed digits are written, numbered over
// the free levels.
hipError_t launch_strassen_pre(int depth, int variant, bool f64, int side, const float* X, int64_t ldx,
                               const PathTable& rows, const PathTable& cols, float* out, int64_t leaf_rows,
                               int64_t leaf_cols, int64_t ldo, int64_t leaf_stride, hipStream_t st,
                               uint32_t fix = kAllFree);
// Same pre-additions writing k-tiled bf16 hi/lo planes (leaf hi at out +
// leaf * leaf_stride, lo at + lo_off; row length ldo, a multiple of 16;
// plane_rows(leaf_rows) rows); f16_scale: fp16 planes, leaf row x multiplied
// by f16_scale[x] first.  side 0: X = A with rows/cols its row and k
// paths.  side 2: X = B (k x n, read in place) producing B^T leaves, rows
// the n paths and cols the k paths.
hipError_t launch_strassen_pre_planes(int depth, int variant, bool f64, int side, const float* X, int64_t ldx,
                                      const PathTable& rows, const PathTable& cols, uint16_t* out, int64_t leaf_rows,
                                      int64_t ldo, int64_t leaf_stride, int64_t lo_off, hipStream_t st,
                                      const float* f16_scale = nullptr, uint32_t fix = kAllFree);
hipError_t launch_strassen_post(int depth, int variant, bool f64, const float* P, int64_t ldp, int64_t leaf_stride,
                                const PathTable& rows, const PathTable& cols, float* C, int64_t ldc,
                                int64_t leaf_rows, int64_t leaf_cols, hipStream_t st);
// Post-addition of one depth-first round: its 7^bf_levels products (the
// breadth-first levels below the depth-first ones, 0..2) combined, then added
// into each target block of C (rows / cols: the full-depth path tables).
hipError_t launch_strassen_post_round(int bf_levels, int variant, bool f64, const float* P, int64_t ldp,
                                      int64_t leaf_stride, const PathTable& rows, const PathTable& cols, float* C,
                                      int64_t ldc, int64_t leaf_rows, int64_t leaf_cols, const RoundTargets& tg,
                                      hipStream_t st);

// Leaf products of a Strassen recursion (or the whole product at depth 0):
// `batch` products of shape m x n x k with the given element strides, run
// by the base kernel of `prec`.  overwrite: C = product, else C += product.
hipError_t launch_base_products(mm_precision prec, int32_t tile, int32_t split_k, int64_t m, int64_t n, int64_t k,
                                const void* A, int64_t lda, int64_t stride_a, const void* B, int64_t ldb,
                                int64_t stride_b, float* C, int64_t ldc, int64_t stride_c, int64_t batch,
                                bool overwrite, float* temps, hipStream_t st, bool planes = false,
                                int64_t a_plane = 0, int64_t b_plane = 0, const float* row_unscale = nullptr,
                                const float* col_unscale = nullptr);

// Workspace bytes the k-split temporaries of `batch` leaf products need.
int64_t base_products_temp_bytes(mm_precision prec, int32_t tile, int32_t split_k, int64_t m, int64_t n, int64_t k,
                                 int64_t batch);

// Strassen product through a schedule (tile / split_k of the leaf products;
// df of the depth levels, counted from the top, depth-first).
mm_status strassen_run(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B, int64_t ldb,
                       float* C, int64_t ldc, int32_t depth, mm_strassen_variant variant, mm_precision prec,
                       int32_t tile, int32_t split_k, int32_t df, void* workspace, size_t workspace_bytes,
                       hipStream_t st);
int64_t strassen_ws_bytes(int64_t m, int64_t n, int64_t k, int32_t depth, mm_precision prec, int32_t tile,
                          int32_t split_k, int32_t df);
// STAR-Strassen (Thm. star-strassen-1): `top` 8-way levels (C blocks x
// k-slices, sub-products serialised in k order) above `depth` Strassen
// levels; one workspace serves every sub-product in turn.
mm_status star_strassen_run(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B,
                            int64_t ldb, float* C, int64_t ldc, int32_t top, int32_t depth,
                            mm_strassen_variant variant, mm_precision prec, int32_t tile, int32_t split_k,
                            int32_t df, void* workspace, size_t workspace_bytes, hipStream_t st);
int64_t star_strassen_ws_bytes(int64_t m, int64_t n, int64_t k, int32_t top, int32_t depth, mm_precision prec,
                               int32_t tile, int32_t split_k, int32_t df);
// The fewest depth-first levels on top (0..depth) whose workspace fits the
// budget, or -1 if none does.
int32_t strassen_choose_df(int64_t m, int64_t n, int64_t k, int32_t top, int32_t depth, mm_precision prec,
                           int32_t tile, int32_t split_k, size_t budget);

}  // namespace starmm
