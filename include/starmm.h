/*
 * starmm: space-bounded divide-and-conquer matrix multiplication on MI355X (gfx950).
 *
 * C ABI of the library.  All matrix pointers are device pointers owned by the
 * caller; every call validates its arguments on the host before it enqueues
 * anything and, on error, enqueues nothing and writes nothing.  Calls are
 * asynchronous on the given HIP stream (a hipStream_t passed as void*; NULL
 * is the default stream), return once the work is enqueued, and keep no
 * reference to any argument after they return.  The only device memory a
 * call may touch besides A, B and C is workspace[0, workspace_bytes): the
 * caller's space budget (mm_semiring_static: the library's static scratch
 * array instead).  A workspace of nonzero size must start at a 256-byte
 * aligned address (hipMalloc and torch allocations do); any other pointer
 * is refused with MM_ERR_INVALID_ARG.  The library allocates no device
 * memory on any of these paths.
 *
 * The method follows Tang, "Improving the Space-Time Efficiency of
 * Processor-Oblivious Matrix Multiplication Algorithms" (arXiv:1911.05328):
 * the semiring product (Sec. 1, eq. mm-dac), its 8-way recursion with
 * k-halves sent to temporaries under a space budget (Sec. mm: CO2, CO3, TAR,
 * SAR, STAR), and Strassen levels (Sec. strassen).
 */
#ifndef STARMM_H
#define STARMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes.  MM_ERR_HIP: a HIP call failed (the message of the last such
 * failure is available from mm_last_error()).  MM_ERR_INCOMPLETE: reported
 * by mm_persistent_status() only. */
typedef enum {
    MM_OK = 0,
    MM_ERR_INVALID_ARG = -1,
    MM_ERR_UNSUPPORTED = -2,
    MM_ERR_WORKSPACE = -3,
    MM_ERR_HIP = -4,
    MM_ERR_INCOMPLETE = -5
} mm_status;

/* The closed semiring (S, (+), (x), 0, 1) of Sec. 1.
 *  MM_SR_PLUS_TIMES: ordinary arithmetic.
 *  MM_SR_MIN_PLUS:   (+) = min, (x) = saturating +, 0 = +INF = 2^30, 1 = 0.
 *                    int32 entries must lie in [0, 2^30]; 2^30 is +INF.
 *  MM_SR_MAX_PLUS:   (+) = max, (x) = saturating +, 0 = -INF = -2^30, 1 = 0.
 *                    int32 entries must lie in [-2^30, 0]; -2^30 is -INF.
 * (x) is saturating: x (x) y = INF when either operand is INF, otherwise
 * x + y clamped to INF.
 *  MM_SR_MAX_MIN:    bottleneck / widest paths: (+) = max, (x) = min,
 *                    0 = INT32_MIN, 1 = INT32_MAX; every int32 is allowed.
 *  MM_SR_OR_AND:     Boolean: (+) = or, (x) = and, 0 = 0, 1 = 1; int32
 *                    entries must be 0 or 1.
 * The integer semirings need int32 A, B, C (MM_DT_I32) and have no Strassen
 * levels (no additive inverse).  Inside these domains the result is exact;
 * entries outside them are a precondition violation (results unspecified,
 * no fault). */
typedef enum {
    MM_SR_PLUS_TIMES = 0,
    MM_SR_MIN_PLUS = 1,
    MM_SR_MAX_PLUS = 2,
    MM_SR_MAX_MIN = 3,
    MM_SR_OR_AND = 4,
    /* range markers: any int32 is a value of the type, so an unknown value
     * passed by a caller is refused by validation, not undefined behaviour */
    MM_SR_RANGE_MIN_ = -2147483647 - 1,
    MM_SR_RANGE_MAX_ = 2147483647
} mm_semiring_kind;

/* Element types.  I32 for the integer semirings (A, B, C all int32).  F32:
 * A, B, C float.  BF16: A, B bfloat16, C float (fp32 accumulation).  F16:
 * A, B IEEE binary16, C float (fp16 MFMA, fp32 accumulation; precision
 * MM_PREC_F32 in the schedule, no Strassen levels). */
typedef enum {
    MM_DT_I32 = 0,
    MM_DT_F32 = 1,
    MM_DT_BF16 = 2,
    MM_DT_F16 = 3,
    MM_DT_RANGE_MIN_ = -2147483647 - 1, /* range markers, as for mm_semiring_kind */
    MM_DT_RANGE_MAX_ = 2147483647
} mm_dtype;

/* Arithmetic of the (+,x) float path.
 *  MM_PREC_F32:    fp32 MFMA products, fp32 accumulation.
 *  MM_PREC_BF16X3: each fp32 operand x is split into hi = bf16(x) and
 *                  lo = bf16(x - hi) (round to nearest even); the product is
 *                  Ah*Bl + Al*Bh + Ah*Bh on bf16 MFMA with fp32 accumulation.
 *                  When the workspace holds them, the split operands are
 *                  first written as bf16 planes (about (m + n) * k * 4 bytes:
 *                  rows rounded up to 32, k to 32; B transposed) and the tile
 *                  kernel copies them; otherwise (or with
 *                  MM_FLAG_SPLIT_IN_KERNEL) the tile kernel splits while
 *                  staging.  Same result either way.
 *  MM_PREC_BF16X3_HIACC: as BF16X3, and the Strassen pre-additions (formed
 *                  from the fp32 inputs) and post-additions are carried out
 *                  in fp64, with one rounding to fp32 at the end.
 *  MM_PREC_BF16:   inputs already bf16 (MM_DT_BF16), one bf16 product.
 *  MM_PREC_FP16X3: the same three products on fp16 MFMA with fp16 hi/lo
 *                  (22 significant bits instead of 16).  fp16's range is
 *                  narrow, so each row i of A (of every Strassen leaf
 *                  operand) is first multiplied by an exact power of two
 *                  s_i and each column j of B by t_j, chosen from the
 *                  largest |entry| of the row / column so that the
 *                  (pre-added) values stay below 2^14; the product is
 *                  multiplied by 1 / (s_i t_j) as it is written.  Needs the
 *                  plane workspace (no in-kernel variant): served by the
 *                  mm_strassen path at every depth, including 0.
 *  MM_PREC_FP16X3_HIACC: FP16X3 with the fp64 Strassen additions of
 *                  BF16X3_HIACC. */
typedef enum {
    MM_PREC_F32 = 0,
    MM_PREC_BF16X3 = 1,
    MM_PREC_BF16X3_HIACC = 2,
    MM_PREC_BF16 = 3,
    MM_PREC_FP16X3 = 4,
    MM_PREC_FP16X3_HIACC = 5,
    MM_PREC_RANGE_MIN_ = -2147483647 - 1, /* range markers, as for mm_semiring_kind */
    MM_PREC_RANGE_MAX_ = 2147483647
} mm_precision;

/* Strassen variants (Sec. strassen).  CLASSIC: the seven products as the
 * paper prints them.  WINOGRAD: Strassen-Winograd, 7 products and 15
 * additions per level. */
typedef enum {
    MM_STRASSEN_CLASSIC = 0,
    MM_STRASSEN_WINOGRAD = 1,
    MM_STRASSEN_RANGE_MIN_ = -2147483647 - 1, /* range markers, as for mm_semiring_kind */
    MM_STRASSEN_RANGE_MAX_ = 2147483647
} mm_strassen_variant;

/*
 * A schedule: how the recursion is flattened onto the GPU.
 *  tile            edge of the square output tile one workgroup owns: the
 *                  base case of the recursion (32, 64 or 128; 256 as well
 *                  for the bf16 / fp16 MFMA kernels).  0 = planner.
 *  split_k         s, the number of k-slices (a power of two, 1..64): the top
 *                  log2(s) recursion levels split k into halves whose
 *                  products run concurrently.  0 = planner.
 *  star_depth      how many of those top levels merge TAR-style (Sec. tar-mm:
 *                  concurrent writes to C serialised by atomic (+), no
 *                  temporaries); the remaining log2(s) - star_depth levels
 *                  merge SAR/CO3-style (the k-half-1 product goes to a
 *                  temporary, merged by madd in a fixed order).  This is the
 *                  STAR hybrid of Sec. star-mm.  Atomic merging is exact for
 *                  (min,+)/(max,+); for floats it needs MM_FLAG_NONDETERMINISTIC.
 *                  With strassen_depth > 0 (or FP16X3) it means something
 *                  else: the number (0..3) of 8-way levels above the Strassen
 *                  levels, the STAR-Strassen hybrid of Thm. star-strassen-1.
 *                  C is split into 2^t x 2^t blocks and k into 2^t slices;
 *                  the 8^t sub-products C_IJ += A_IL B_LJ (L ascending,
 *                  blocks in recursion order) each run the Strassen levels
 *                  in turn on the stream, reusing one workspace sized for
 *                  the largest sub-product (about 4^-t of the Strassen
 *                  workspace), for 8^t times more, smaller launches.
 *                  Results are deterministic.
 *  strassen_depth  Strassen levels above the base product ((+,x) only, 0..3).
 *  strassen_layout how the Strassen levels hold their temporaries.  0 = the
 *                  planner: every level breadth-first when the workspace
 *                  holds it, else the fewest depth-first levels on top that
 *                  fit.  MM_STRASSEN_LAYOUT(mask): bit l set makes level l
 *                  (0 = the top) depth-first, clear makes it breadth-first.
 *                  A breadth-first level forms the operands of its seven
 *                  products at once and runs them together (the
 *                  straightforward parallel Strassen of Lemma par-strassen:
 *                  workspace grows by 7/4 per level).  A depth-first level
 *                  takes its seven products one after another, forming S_r
 *                  and T_r on the fly from A and B and adding the product
 *                  into C at once (SAR-Strassen, Lemma sar-strassen), so the
 *                  temporaries of one product are reused by the next: with
 *                  the top t levels depth-first a product takes 7^t rounds,
 *                  each forming and multiplying the 7^(depth - t) leaves of
 *                  the breadth-first levels below, and the workspace is that
 *                  of one round.  Depth-first levels must be the top ones
 *                  (mask = 2^t - 1; others are MM_ERR_UNSUPPORTED).  Results
 *                  are deterministic; the rounding order of the additions
 *                  depends on the layout.
 *  variant         mm_strassen_variant.
 *  precision       mm_precision of the float path.
 *  band_rows       rows of C processed per pass; the temporaries of one pass
 *                  are reused by the next, so the space is bounded by the
 *                  band rather than by C (the memory-reuse argument of
 *                  Sec. sar-mm).  0 = all rows in one pass, or the largest
 *                  band the workspace allows when the planner chooses.
 *  flags           MM_FLAG_*.
 */
typedef struct {
    int32_t tile;
    int32_t split_k;
    int32_t star_depth;
    int32_t strassen_depth;
    int32_t variant;
    int32_t precision;
    int64_t band_rows;
    int32_t flags;
    int32_t strassen_layout;
} mm_schedule;

#define MM_STRASSEN_LAYOUT_GIVEN 0x100
#define MM_STRASSEN_LAYOUT(depth_first_mask) (MM_STRASSEN_LAYOUT_GIVEN | (depth_first_mask))

#define MM_FLAG_NONDETERMINISTIC 1 /* allow float atomics (run-to-run rounding differences) */
#define MM_FLAG_SPLIT_IN_KERNEL 2  /* BF16x3: never use workspace for pre-split operand planes */
/* Integer semirings: one persistent launch whose resident workgroups take
 * (tile, k-slice) items in order; the partial results of a tile's slices go
 * to a ring of slot groups whose size does not depend on the problem
 * (MM_PERSIST_SLOTS tiles of partials in all, rounded to whole groups of
 * split_k; one group per output tile when there are fewer tiles), and the
 * slice that arrives last merges them into C in slice order.  A tile waits
 * for its group only until the group's previous tile has been merged; every
 * such wait ends (items go out in order to running workgroups), and it is
 * also bounded by a spin count scaled with the k-depth of a slice.  A wait
 * that exceeds the bound leaves C incomplete and sets an error word in the
 * workspace's control block, which mm_persistent_status() reports.  With
 * split_k = 1 no slots are used.  Needs star_depth 0 and band_rows 0. */
#define MM_FLAG_PERSISTENT 4
#define MM_PERSIST_SLOTS 2048
/* Integer semirings, wider input domain (the fast path's precondition is
 * (min,+) entries in [0, 2^30], (max,+) entries in [-2^30, 0]): (min,+)
 * entries anywhere in [-2^30, 2^30] (2^30 = +INF; an INF operand gives INF
 * whatever its partner, and a sum >= 2^30 gives INF), results in
 * [-2^31, 2^30]; (max,+) entries in [-2^30, 2^30 - 1] (-2^30 = -INF), results
 * in [-2^30, 2^31 - 2].  Same speed class as the fast path (operands are
 * shifted on load and multiplied with a saturating add).  Accepted and
 * without effect for (max, min), which takes every int32 anyway;
 * MM_ERR_INVALID_ARG for (+,x) and Boolean. */
#define MM_FLAG_CHECKED_RANGE 8
/* mm_batched only: C = A B for this problem (C is written, never read)
 * instead of C += A B.  MM_ERR_INVALID_ARG elsewhere. */
#define MM_FLAG_OVERWRITE_C 16

/*
 * The plan the library derives from (problem, schedule, budget).  Exported
 * for inspection and tests; filled by mm_plan().
 */
typedef struct {
    mm_schedule sched;         /* the resolved schedule (no zeros left) */
    int32_t tile_k;            /* k-depth of one staged tile */
    int32_t tar_levels;        /* = sched.star_depth (with Strassen: 8-way levels above) */
    int32_t sar_levels;        /* log2(split_k) - star_depth */
    int64_t bands;             /* number of passes over C */
    int64_t tiles_m, tiles_n;  /* output tiles per band row / column */
    int64_t workgroups;        /* workgroups of the main launch (one band); (tile, slice)
                                  items of a persistent launch */
    int64_t temp_elems;        /* temporary C elements (per band, all groups) */
    int64_t ws_bytes;          /* workspace bytes the plan uses */
    int64_t leaf_m, leaf_n, leaf_k; /* base product dims after Strassen levels */
    int64_t leaves;            /* 8^(8-way levels above Strassen) x 7^strassen_depth */
} mm_plan_info;

/*
 * C <- C (+) A (x) B   (Sec. 1, eq. mm-dac; base kernels accumulate into C
 * because both k-halves update the same quadrant, Fig. mm-n2).
 *
 * A is m x k (row-major, leading dimension lda >= k), B is k x n (ldb >= n),
 * C is m x n (ldc >= n), all device memory of type dt (C is float for BF16
 * and F16).  Semirings: MIN_PLUS, MAX_PLUS, MAX_MIN and OR_AND need
 * dt = I32; PLUS_TIMES needs F32, BF16 or F16.
 * sched == NULL lets the planner choose (or the loaded timings and cost
 * model, see mm_tuned_load), never exceeding workspace_bytes; an
 * explicit schedule that does not fit returns MM_ERR_WORKSPACE.  A schedule
 * with strassen_depth > 0 on a non-ring semiring returns MM_ERR_UNSUPPORTED
 * (Strassen needs the inverse of (+), Sec. strassen).
 * m, n or k == 0 is valid (k == 0 leaves C unchanged): such a product
 * launches nothing and needs no workspace, whatever the schedule (operand
 * pointers of empty matrices may be NULL).
 */
mm_status mm_semiring(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                      const void *A, int64_t lda, const void *B, int64_t ldb,
                      void *C, int64_t ldc, void *workspace, size_t workspace_bytes,
                      const mm_schedule *sched, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as mm_semiring, with the library's own static scratch array as the
 * workspace instead of a caller buffer.  The array is a file-scope device
 * array of MM_STATIC_SCRATCH_BYTES (64 MiB) plus 256 bytes, one copy on each
 * GPU the library runs on, held until the process ends; its address is
 * looked up on the first call on each device.  The call allocates nothing
 * (no hipMalloc / hipFree; the STARMM_CHECK_DOMAIN debugging mode counts
 * into the array's first word).
 *  sched == NULL: the built-in planner with a budget of
 *    MM_STATIC_SCRATCH_BYTES (the loaded timings / cost model of
 *    mm_tuned_load are not consulted).
 *  An explicit schedule needing more than MM_STATIC_SCRATCH_BYTES returns
 *  MM_ERR_WORKSPACE (mm_last_error() names the need), launching nothing;
 *  MM_FLAG_PERSISTENT returns MM_ERR_UNSUPPORTED (its status word would have
 *  no caller-visible home).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind; a call initialises what it reads (temporaries are overwritten by
 * their first k-tile, planes and counters are rewritten by its kernels).
 * Calls on one stream are ordered; two calls that overlap in time on one GPU
 * (other streams, other threads) race on the array and their results are
 * undefined.  Otherwise arguments, validation and errors as mm_semiring.
 */
#define MM_STATIC_SCRATCH_BYTES (64u << 20)
mm_status mm_semiring_static(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                             const void *A, int64_t lda, const void *B, int64_t ldb,
                             void *C, int64_t ldc, const mm_schedule *sched, void *stream);

/*
 * C <- C + A B over fp32 by `depth` levels of Strassen (Sec. strassen;
 * variant MM_STRASSEN_CLASSIC is the seven products as printed,
 * MM_STRASSEN_WINOGRAD is Strassen-Winograd) above a base GEMM of precision
 * `prec` (MM_PREC_F32, MM_PREC_BF16X3, MM_PREC_BF16X3_HIACC, MM_PREC_FP16X3 or
 * MM_PREC_FP16X3_HIACC).
 * When the workspace holds it, all levels are breadth-first: the operands of
 * all 7^depth base products are formed first (the straightforward parallel
 * Strassen of Lemma par-strassen), so workspace grows as (7/4)^depth times
 * the inputs; see mm_strassen_workspace_bytes().  A smaller workspace makes
 * the fewest top levels depth-first that fit (SAR-Strassen, Lemma
 * sar-strassen; see strassen_layout in mm_schedule); MM_ERR_WORKSPACE only
 * when even every level depth-first does not fit (mm_workspace_bytes with
 * a schedule of strassen_layout MM_STRASSEN_LAYOUT(2^depth - 1) tells that
 * size).  depth 0..3.  Matrix layout as in mm_semiring; m, n or k == 0
 * launches nothing and needs no workspace (k == 0 leaves C unchanged).
 */
mm_status mm_strassen(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda,
                      const float *B, int64_t ldb, float *C, int64_t ldc,
                      int32_t depth, mm_strassen_variant variant, mm_precision prec,
                      void *workspace, size_t workspace_bytes, void *stream);

/*
 * The coefficients one Strassen level uses (Sec. strassen): for product r
 * (0..6) and quadrant (i, j), alpha[r*4 + i*2 + j] is the coefficient of A_ij
 * in the A-side operand, beta of B_ij in the B-side operand, gamma of P_r in
 * C_ij.  Arrays of 28 int8 each, caller-owned.  Pure host code.
 */
mm_status mm_strassen_coefficients(mm_strassen_variant variant, int8_t *alpha, int8_t *beta, int8_t *gamma);

/*
 * General bilinear schemes (the bilinear-circuit form of Strassen-like
 * algorithms in the closing remarks of Sec. strassen, eq. bilinear).  A
 * scheme on a g x g block grid with R products:
 *   product r multiplies S_r = sum_p alpha[r*g*g + p] A_p by
 *   T_r = sum_q beta[r*g*g + q] B_q, and C_c gains sum_r gamma[c*R + r] P_r,
 * with block indices p = i*g + l (A: block-row i, block-column l),
 * q = l*g + j (B) and c = i*g + j (C).  Only the first R*g*g (g*g*R) entries
 * of each array are read.
 */
#define MM_BILINEAR_MAX_GRID 4
#define MM_BILINEAR_MAX_PRODUCTS 64
typedef struct {
    int32_t g;        /* grid edge, 1..MM_BILINEAR_MAX_GRID */
    int32_t products; /* R, 1..MM_BILINEAR_MAX_PRODUCTS */
    int8_t alpha[MM_BILINEAR_MAX_PRODUCTS * MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_GRID];
    int8_t beta[MM_BILINEAR_MAX_PRODUCTS * MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_GRID];
    int8_t gamma[MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_PRODUCTS];
} mm_bilinear_scheme;

/* Built-in schemes (pure host code): MM_BILINEAR_CLASSICAL with param = g
 * (1..4; the g^3 block products of the definition) and
 * MM_BILINEAR_STRASSEN with param = an mm_strassen_variant (the seven
 * products of mm_strassen_coefficients on the 2 x 2 grid).
 * MM_ERR_INVALID_ARG on other kinds or params. */
typedef enum {
    MM_BILINEAR_CLASSICAL = 0,
    MM_BILINEAR_STRASSEN = 1,
    MM_BILINEAR_RANGE_MIN_ = INT32_MIN, MM_BILINEAR_RANGE_MAX_ = INT32_MAX
} mm_bilinear_kind;
mm_status mm_bilinear_builtin(mm_bilinear_kind kind, int32_t param, mm_bilinear_scheme *out);

/* The scheme that applies s1 to the g1 x g1 grid and s2 inside each block,
 * as one level on the (g1 g2) x (g1 g2) grid: block index i = i1*g2 + i2,
 * product r = r1*R2 + r2, coefficients multiplied.  MM_ERR_INVALID_ARG if
 * g1 g2 > MM_BILINEAR_MAX_GRID, R1 R2 > MM_BILINEAR_MAX_PRODUCTS or a
 * coefficient leaves int8.  Pure host code. */
mm_status mm_bilinear_product(const mm_bilinear_scheme *s1, const mm_bilinear_scheme *s2, mm_bilinear_scheme *out);

/* MM_OK if the scheme multiplies matrices: its coefficients reproduce the
 * matrix multiplication tensor, sum_r alpha[r,(i,l)] beta[r,(l',j)]
 * gamma[(i',j'),r] = [i = i'][l = l'][j = j'] for every index; else
 * MM_ERR_INVALID_ARG.  Pure host code. */
mm_status mm_bilinear_scheme_check(const mm_bilinear_scheme *s);

/* Workspace bytes of mm_bilinear (0 on invalid arguments or an empty
 * product). */
size_t mm_bilinear_workspace_bytes(int64_t m, int64_t n, int64_t k, const mm_bilinear_scheme *s,
                                   mm_precision prec);

/*
 * C <- C + A B over fp32 through one level of the bilinear scheme s above
 * the BF16x3 base product (prec must be MM_PREC_BF16X3; others return
 * MM_ERR_UNSUPPORTED).  A, B and C are cut into g x g grids of blocks of
 * ceil(m/g) x ceil(k/g), ceil(k/g) x ceil(n/g) and ceil(m/g) x ceil(n/g),
 * zero-padded at the edges (exact over a ring).  The operand sums S_r and
 * T_r are formed in fp32 in ascending block order straight into k-tiled
 * bf16 hi/lo planes, the R products run as one batched launch of the
 * base-product tiles, and the output sums in fp32 in ascending product
 * order, so results are deterministic.  The scheme must pass
 * mm_bilinear_scheme_check (else MM_ERR_INVALID_ARG).  Workspace: at least
 * mm_bilinear_workspace_bytes() (else MM_ERR_WORKSPACE); m, n or k == 0
 * launches nothing.  Matrix layout as in mm_semiring.
 */
mm_status mm_bilinear(int64_t m, int64_t n, int64_t k, const float *A, int64_t lda, const float *B,
                      int64_t ldb, float *C, int64_t ldc, const mm_bilinear_scheme *s, mm_precision prec,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes mm_strassen needs for these arguments with every level
 * breadth-first, its fastest layout (0 on invalid ones). */
size_t mm_strassen_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t depth,
                                   mm_strassen_variant variant, mm_precision prec);

/*
 * Plan only (pure host code, no HIP call): resolve `sched` (NULL = planner)
 * for this problem and budget.  Returns the status mm_semiring would return
 * for these arguments before any launch.
 */
mm_status mm_plan(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                  size_t workspace_bytes, const mm_schedule *sched, mm_plan_info *out);

/* Workspace bytes mm_semiring needs for this schedule (NULL = the built-in
 * planner's choice with an unlimited budget). */
size_t mm_workspace_bytes(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                          const mm_schedule *sched);

/*
 * Outcome of the last persistent (MM_FLAG_PERSISTENT) mm_semiring call that
 * used this workspace: waits for `stream`, then reads the control block's
 * error word (the first bytes of the workspace).  MM_OK: every bounded wait
 * ended normally and C is complete.  MM_ERR_INCOMPLETE: a wait exceeded its
 * bound and C is incomplete (the call itself had returned MM_OK, since it
 * returns once the work is enqueued).  MM_ERR_INVALID_ARG: null workspace or
 * fewer bytes than the control block (256).  MM_ERR_HIP: the copy or the
 * wait failed.  Synchronising: not for graph capture.
 */
mm_status mm_persistent_status(const void *workspace, size_t workspace_bytes, void *stream);

/* Static text for a status code. */
const char *mm_status_string(mm_status st);

/* Text of the last HIP failure on this thread ("" if none). */
const char *mm_last_error(void);

/*
 * One (+,x) product of a batch: C (m x n, float) += A (m x k) B (k x n),
 * row-major with leading dimensions; device pointers owned by the caller.
 */
typedef struct {
    int64_t m, n, k;
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    float *C;
    int64_t ldc;
} mm_problem;

/*
 * Many independent products of uneven shape in ONE persistent kernel launch
 * (the flattened recursion's base-case tiles of every problem form one work
 * list, handed out longest-first by a device counter).  dt = MM_DT_BF16: A, B
 * bfloat16, one bf16 product, fp32 accumulation (MM_DT_F16: fp16 the same
 * way, fp16 MFMA).  dt = MM_DT_F32: A, B float,
 * BF16x3 split product.  scheds (NULL or one per problem): split_k per problem
 * (power of two <= 64; partial tiles go to workspace slots and the last slice
 * to arrive sums them in ascending slice order, so results are deterministic);
 * tile 0, 128 or 256 (256 needs the packed planes); strassen_depth > 0 is
 * MM_ERR_UNSUPPORTED; flags: MM_FLAG_SPLIT_IN_KERNEL and / or
 * MM_FLAG_OVERWRITE_C (C = A B with plain stores: C is not read, which halves
 * the C traffic and needs no atomics).  By default a pack kernel first rewrites each
 * problem's A and B^T into k-tiled 16-bit planes in the workspace (hi/lo for
 * MM_DT_F32), so tiles stage aligned 16-byte chunks whatever the strides;
 * MM_FLAG_SPLIT_IN_KERNEL on a problem stages it straight from its operands
 * (no plane space).  Problems must not overlap in C.  The workspace holds
 * the problem table, the work list, counters, slots and planes:
 * mm_batched_workspace_bytes() tells the size (MM_ERR_WORKSPACE if smaller).
 * The tables are copied from host memory during the call (stream-ordered).
 */
size_t mm_batched_workspace_bytes(int32_t count, const mm_problem *problems, mm_dtype dt,
                                  const mm_schedule *scheds);
mm_status mm_batched(int32_t count, const mm_problem *problems, mm_dtype dt,
                     const mm_schedule *scheds, void *workspace, size_t workspace_bytes,
                     void *stream);

/*
 * The same batch captured once in a hipGraph holding the pack kernel and the
 * persistent kernel, then replayed with mm_batched_graph_launch() on any
 * stream (every replay repacks, so operand updates between replays count).  Create
 * uploads the tables into the workspace and waits for that upload; the
 * workspace and every problem's buffers must stay valid and the workspace
 * untouched by others until mm_batched_graph_destroy().  Replays on one
 * workspace must not overlap in time (they share its counters).
 */
typedef struct mm_batched_graph mm_batched_graph;
mm_status mm_batched_graph_create(int32_t count, const mm_problem *problems, mm_dtype dt,
                                  const mm_schedule *scheds, void *workspace,
                                  size_t workspace_bytes, void *stream, mm_batched_graph **out);
mm_status mm_batched_graph_launch(mm_batched_graph *g, void *stream);
void mm_batched_graph_destroy(mm_batched_graph *g);

/*
 * Kernels of the schedule cost model (a small MLP trained on the GPU; not in
 * the paper).  All buffers are device float32, row-major, caller-owned.
 *
 * mm_mlp_linear_forward: Y[b,o] = act(sum_i X[b,i] W[o,i] + bias[o]) for
 *   X batch x in, W out x in, bias out (may be NULL), Y batch x out;
 *   act = ReLU if relu != 0, else identity.
 * mm_mlp_linear_backward: for the same layer, given its output Y and dL/dY:
 *   dZ = dY * [Y > 0] (ReLU) or dY (batch x out, scratch the caller provides),
 *   dX = dZ W (batch x in; skipped if dX is NULL), dW = dZ^T X (out x in),
 *   db = column sums of dZ (skipped if db is NULL).
 * mm_mlp_masked_mse: over `total` elements, loss = sum M (P - T)^2 /
 *   max(1, sum M) written to *loss (device scalar, may be NULL) and
 *   dP = 2 M (P - T) / max(1, sum M) (may be NULL).
 * mm_mlp_adam: Adam update of `count` parameters with bias correction for
 *   step >= 1: m1 = b1 m1 + (1-b1) g, m2 = b2 m2 + (1-b2) g^2,
 *   param -= lr (m1 / (1 - b1^step)) / (sqrt(m2 / (1 - b2^step)) + eps).
 * Every reduction runs in a fixed order (bitwise reproducible).
 */
mm_status mm_mlp_linear_forward(int64_t batch, int64_t in, int64_t out, const float *X, const float *W,
                                const float *bias, float *Y, int32_t relu, void *stream);
mm_status mm_mlp_linear_backward(int64_t batch, int64_t in, int64_t out, const float *X, const float *W,
                                 const float *Y, const float *dY, float *dZ, float *dX, float *dW, float *db,
                                 int32_t relu, void *stream);
mm_status mm_mlp_masked_mse(int64_t total, const float *P, const float *T, const float *M, float *loss,
                            float *dP, void *stream);
mm_status mm_mlp_adam(int64_t count, float *param, const float *grad, float *m1, float *m2, float lr,
                      float beta1, float beta2, float eps, int32_t step, void *stream);

/*
 * Per-kernel timing for measurement.  mm_profile_enable(1) makes every
 * subsequent kernel launch of the library record a HIP event before and
 * after it on its own stream.  mm_profile_summary() waits for the recorded
 * events and writes a JSON object {"<kernel family>": [launches, total_ms],
 * ...} into buf (truncated to len-1 bytes, NUL-terminated); it returns the
 * full length.  mm_profile_reset() forgets the records.  Not thread-safe
 * against concurrent launches from other threads.
 */
void mm_profile_enable(int32_t on);
void mm_profile_reset(void);
int64_t mm_profile_summary(char *buf, size_t len);

/*
 * Microbenchmarks of the achievable peaks the kernels are bounded by
 * (measurement only).  kind 0: int32 add / min VALU loop (work = lane-ops);
 * 1: bf16 32x32x16 MFMA loop (flops); 2: fp32 32x32x2 MFMA loop (flops);
 * 3: device copy of `bytes` from buf_a to buf_b (work = bytes read + written).
 * Kinds 0-2 take `iters` loop steps and need buf_a to hold one 4-byte word per
 * workgroup (8 x CUs).  Enqueues one kernel on `stream` and stores the work
 * it performs in *work; the caller times it.
 */
mm_status mm_microbench(int32_t kind, int64_t iters, void *buf_a, void *buf_b, int64_t bytes, double *work,
                        void *stream);

/* Library version as major*10000 + minor*100 + patch. */
int32_t mm_version(void);

/*
 * The order in which the tile kernels visit a grid of tm x tn output tiles
 * (the flattened recursion of eq. mm-dac: quadrants 00, 01, 10, 11 for
 * square-ish grids, halving only the long side of a grid at least twice as
 * long as wide): the t-th visited tile is (ti[t], tj[t]), t < tm * tn.
 * Host memory owned by the caller; pure host code (no GPU needed).
 * MM_ERR_INVALID_ARG for negative sizes, null outputs with tiles to write,
 * or more than 2^26 tiles.
 */
mm_status mm_tile_order(int64_t tm, int64_t tn, int64_t *ti, int64_t *tj);

/*
 * Input-domain check for the integer semirings (a debugging aid; the fast
 * paths do not test their inputs, Sec. 1's semirings carry no infinities and
 * the sentinel arithmetic is this library's): writes to *count (one device
 * uint64, caller-owned) the number of entries of X (rows x cols int32,
 * row-major, leading dimension ld >= cols, device memory) outside the domain
 * mm_semiring assumes for (sr, flags): (min,+) [0, 2^30], or [-2^30, 2^30]
 * with MM_FLAG_CHECKED_RANGE; (max,+) [-2^30, 0], or [-2^30, 2^30 - 1];
 * Boolean {0, 1}; (max, min) has none (always 0).  Asynchronous on stream.
 * MM_ERR_INVALID_ARG for (+,x), unknown flags, negative sizes, ld < cols, a
 * null count, or a null X with entries.
 *
 * With the environment variable STARMM_CHECK_DOMAIN set (to anything but
 * "0"), every integer-semiring mm_semiring call runs this check on A, B and
 * C first, waits for it (synchronising the stream) and returns
 * MM_ERR_INVALID_ARG, launching nothing, if any entry is outside; the
 * counter it uses is one word of device memory per device, allocated on the
 * first checked call and kept until the process ends.
 */
mm_status mm_domain_violations(mm_semiring_kind sr, int32_t flags, const int32_t *X, int64_t rows, int64_t cols,
                               int64_t ld, unsigned long long *count, void *stream);

/*
 * Schedule selection for calls without a schedule (the autotuner and its
 * learned cost model; not part of the paper).  By default mm_semiring and
 * mm_plan with sched == NULL use the built-in planner.  Once timings and/or a
 * cost model are loaded, such a call takes, in this order:
 *   1. the fastest loaded timing for exactly (semiring, dtype, m, n, k) whose
 *      schedule runs within workspace_bytes as it was timed;
 *   2. the cost model's proposal: the schedule of least predicted time among
 *      those of its space (Strassen depth 0-3 x split_k 1, 2, 4, 8 x tile 32,
 *      64, 128, 256) that the planner accepts within workspace_bytes and
 *      whose measured error the model's accuracy mask accepts;
 *   3. the built-in planner.
 * Both are opt-in: the cost model's space computes fp32 products through
 * split precision (MM_PREC_BF16X3 without Strassen levels, MM_PREC_FP16X3
 * under up to three Winograd levels), held to a relative error of 1e-5 by
 * the tuner's measurements rather than to MM_PREC_F32's rounding.  The model covers
 * PLUS_TIMES with F32 or BF16 and MIN_PLUS with I32; other pairs go to the
 * timings or the planner.  mm_workspace_bytes(NULL) keeps reporting the
 * built-in planner's need; every selected schedule fits the budget passed.
 * mm_batched ignores the selection: the timings are of products launched
 * alone, whose k-splits only add merge work in a batch that fills the GPU.  The selection is process-wide state
 * guarded by a lock; loads replace what was loaded before.  Pure host code.
 */

/* One measured timing: problem, schedule (as passed to mm_semiring), time. */
typedef struct {
    int32_t semiring;  /* mm_semiring_kind */
    int32_t dtype;     /* mm_dtype */
    int64_t m, n, k;
    mm_schedule sched;
    double ms;
} mm_tuned_entry;

/* Number of float parameters mm_cost_model_load expects: 13,186 (t_mean,
 * t_std, the 12,992 weights and biases of the 7-64-64-64-64 network, and
 * the 192 entries of the accuracy mask). */
int64_t mm_cost_model_param_count(void);

/*
 * Load the cost model from host memory: t_mean, t_std (the log-time
 * standardisation, t_std > 0), then for each of the four layers its weights
 * (out x in, row-major) and biases, then the accuracy mask: for the space's
 * dtypes fp32, bf16, int32 (min,+) in that order, 64 entries each, 1 when
 * the schedule's measured error stayed within the error target (1e-5
 * relative Frobenius against the float64 product), 0 when the proposal must
 * leave it out.  The library copies them.  MM_ERR_INVALID_ARG for a null
 * pointer, a wrong count, non-finite values or mask entries other than 0 / 1.
 */
mm_status mm_cost_model_load(const float *params, int64_t count);

/* Load measured timings (host memory, copied).  MM_ERR_INVALID_ARG for
 * non-positive sizes, a negative or non-finite time, or a schedule the
 * planner rejects for its problem under any budget; nothing is loaded then. */
mm_status mm_tuned_load(const mm_tuned_entry *entries, int64_t count);

/* Forget the loaded cost model and timings (back to the built-in planner). */
void mm_schedule_selection_clear(void);

/*
 * The cost model's proposal for this problem and budget, with its predicted
 * time in milliseconds (predicted_ms may be NULL).  MM_ERR_UNSUPPORTED
 * without a loaded model or for a (semiring, dtype) pair outside its space;
 * MM_ERR_WORKSPACE when no schedule of the space fits; MM_ERR_INVALID_ARG
 * for a null output or a zero size.
 */
mm_status mm_propose_schedule(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                              size_t workspace_bytes, mm_schedule *out, double *predicted_ms);

/* The fastest loaded timing for exactly this problem that runs within the
 * budget as timed, and its time (measured_ms may be NULL).
 * MM_ERR_UNSUPPORTED when there is none. */
mm_status mm_tuned_lookup(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                          size_t workspace_bytes, mm_schedule *out, double *measured_ms);

#ifdef __cplusplus
}
#endif

#endif /* STARMM_H */
