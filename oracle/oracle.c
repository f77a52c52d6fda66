/*
 * Oracle for the space-bounded divide-and-conquer matrix multiply.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or constant generator with the HIP
 * path.
 *
 * Everything here is plain, slow C in int64 / double, written for a reader
 * who checks it against the paper (Tang, "Improving the Space-Time Efficiency
 * of Processor-Oblivious Matrix Multiplication Algorithms"):
 *   - the semiring product C = A (x) B on (S, (+), (x), 0, 1)   (Sec. 1, eq. mm-dac)
 *   - the 8-way recursion in CO2 order                           (Fig. mm-n2)
 *   - the same recursion with k-halves sent to temporaries and
 *     merged by madd (CO3 / SAR lazy allocation)                 (Fig. mm-n3, Fig. wrapper-sar-mm, Sec. sar-mm)
 *   - Strassen's seven products as printed in the paper          (Sec. strassen)
 *   - Strassen-Winograd (7 products, 15 additions), the textbook
 *     form of the variant the paper names among bilinear schemes (Sec. strassen, closing remarks)
 *
 * Integer semirings use a saturating sentinel: INF = 2^30 for (min,+),
 * -INF = -2^30 for (max,+).  x (x) y is INF when either operand is INF,
 * otherwise x + y clamped to INF.  The paper does not treat infinities; this
 * is the reading the library documents.
 *
 * Two more closed semirings on int32 (the paper's product is stated for any
 * semiring):
 *   - (max, min), the bottleneck / widest-path semiring: (+) = max,
 *     (x) = min, zero = the smallest int32 (annihilates min, neutral under
 *     max), one = the largest;
 *   - Boolean (OR, AND) on {0, 1}: (+) = logical or, (x) = logical and,
 *     zero = 0 (false), one = 1 (true).
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_PLUS_TIMES = 0, OR_MIN_PLUS = 1, OR_MAX_PLUS = 2, OR_MAX_MIN = 3, OR_OR_AND = 4 };
#define OR_I32_MIN (-((int64_t)1 << 31))
#define OR_INF ((int64_t)1 << 30)

/* Threads of the parallel loops (timing the oracle on one core). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- semiring */

static int64_t sr_zero(int sr)
{
    if (sr == OR_MIN_PLUS) return OR_INF;
    if (sr == OR_MAX_PLUS) return -OR_INF;
    if (sr == OR_MAX_MIN) return OR_I32_MIN;
    return 0; /* (+,x) and (or, and) */
}

/* (x): multiplicative operation of the semiring. */
static int64_t sr_mul(int sr, int64_t x, int64_t y)
{
    if (sr == OR_MIN_PLUS) {
        if (x >= OR_INF || y >= OR_INF) return OR_INF;
        int64_t s = x + y;
        return s < OR_INF ? s : OR_INF;
    }
    if (sr == OR_MAX_PLUS) {
        if (x <= -OR_INF || y <= -OR_INF) return -OR_INF;
        int64_t s = x + y;
        return s > -OR_INF ? s : -OR_INF;
    }
    if (sr == OR_MAX_MIN) return x < y ? x : y;
    if (sr == OR_OR_AND) return (x != 0 && y != 0) ? 1 : 0;
    return x * y;
}

/* (+): additive operation of the semiring. */
static int64_t sr_add(int sr, int64_t x, int64_t y)
{
    if (sr == OR_MIN_PLUS) return x < y ? x : y;
    if (sr == OR_MAX_PLUS) return x > y ? x : y;
    if (sr == OR_MAX_MIN) return x > y ? x : y;
    if (sr == OR_OR_AND) return (x != 0 || y != 0) ? 1 : 0;
    return x + y;
}

/* ------------------------------------------------------------- brute force */

/* C_ij <- C_ij (+) (+)_{l<k} A_il (x) B_lj : the definition of the product.
 * Loop order i-l-j: for every (i, j) the terms still join C_ij one at a time
 * in increasing l, as in the definition; the j loop only lets the compiler
 * stream rows of B.  `row_step` applies one l to a row of C for a fixed
 * semiring (constant sr, so the semiring operations inline). */
static void row_step(int sr, int64_t n, int64_t a, const int64_t *b, int64_t *c)
{
    for (int64_t j = 0; j < n; ++j) c[j] = sr_add(sr, c[j], sr_mul(sr, a, b[j]));
}

void or_brute_i64(int sr, int64_t m, int64_t n, int64_t k,
                  const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb,
                  int64_t *C, int64_t ldc)
{
#pragma omp parallel for schedule(static) if (m * n * k > 1000000)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t l = 0; l < k; ++l) {
            const int64_t a = A[i * lda + l];
            const int64_t *b = B + l * ldb;
            int64_t *c = C + i * ldc;
            switch (sr) {
            case OR_MIN_PLUS: row_step(OR_MIN_PLUS, n, a, b, c); break;
            case OR_MAX_PLUS: row_step(OR_MAX_PLUS, n, a, b, c); break;
            case OR_MAX_MIN: row_step(OR_MAX_MIN, n, a, b, c); break;
            case OR_OR_AND: row_step(OR_OR_AND, n, a, b, c); break;
            default: row_step(OR_PLUS_TIMES, n, a, b, c); break;
            }
        }
}

/* Ordinary (+,x) product in double: C <- C + A B.  Loop order i-l-j so the
 * compiler can stream rows of B; the sum over l is taken in increasing l. */
void or_brute_f64(int64_t m, int64_t n, int64_t k,
                  const double *A, int64_t lda, const double *B, int64_t ldb,
                  double *C, int64_t ldc)
{
#pragma omp parallel for schedule(static) if (m * n * k > 1000000)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t l = 0; l < k; ++l) {
            double a = A[i * lda + l];
            const double *b = B + l * ldb;
            double *c = C + i * ldc;
            for (int64_t j = 0; j < n; ++j) c[j] += a * b[j];
        }
}

/* ------------------------------------------------- 8-way recursion (CO2/CO3) */

/*
 * Shared state of one recursive call tree.  `split_mask` bit d set means
 * "at recursion depth d, the k-half-1 sub-products write a temporary D (of
 * the size of the current C block) instead of C itself, and D is merged into
 * C with madd after both halves finish" (CO3 at that depth; the k-half-0
 * products keep working on the parent's storage, which is the paper's lazy
 * allocation).  With split_mask == 0 this is exactly CO2: both k-halves
 * update C one after the other.
 */
typedef struct {
    int sr;
    int64_t b;            /* base case: max(m, n, k) <= b (dimension, not element count) */
    uint32_t split_mask;
    int64_t temp_total;   /* sum of sizes of all temporaries ever requested */
    int64_t temp_live;    /* currently live temporary elements (depth-first run) */
    int64_t temp_peak;    /* peak of temp_live */
    int64_t leaves;       /* number of base-case products */
    int is_f64;
} rec_ctx;

static void rec_i64(rec_ctx *cx, int depth, int64_t m, int64_t n, int64_t k,
                    const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb,
                    int64_t *C, int64_t ldc);

/* C (+)= A (x) B on one block, splitting m, n, k into ceil/floor halves. */
static void rec_i64(rec_ctx *cx, int depth, int64_t m, int64_t n, int64_t k,
                    const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb,
                    int64_t *C, int64_t ldc)
{
    if (m == 0 || n == 0 || k == 0) return;
    int64_t mx = m > n ? m : n;
    if (k > mx) mx = k;
    if (mx <= cx->b) {
        cx->leaves++;
        or_brute_i64(cx->sr, m, n, k, A, lda, B, ldb, C, ldc);
        return;
    }
    int64_t m0 = (m + 1) / 2, n0 = (n + 1) / 2, k0 = (k + 1) / 2;
    int64_t mh[2] = {m0, m - m0}, nh[2] = {n0, n - n0}, kh[2] = {k0, k - k0};
    int split = (cx->split_mask >> depth) & 1u;

    /* Storage that the k-half-1 products update: C itself, or a temporary D. */
    int64_t *D = C;
    int64_t ldd = ldc;
    if (split) {
        D = (int64_t *)malloc((size_t)(m * n) * sizeof(int64_t));
        ldd = n;
        int64_t z = sr_zero(cx->sr);
        for (int64_t t = 0; t < m * n; ++t) D[t] = z;
        cx->temp_total += m * n;
        cx->temp_live += m * n;
        if (cx->temp_live > cx->temp_peak) cx->temp_peak = cx->temp_live;
    }
    /* eq. (mm-dac): C_ij (+)= A_i0 (x) B_0j, then C_ij (+)= A_i1 (x) B_1j. */
    for (int h = 0; h < 2; ++h) {
        int64_t *T = h == 0 ? C : D;
        int64_t ldt = h == 0 ? ldc : ldd;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const int64_t *Aih = A + (i ? m0 : 0) * lda + (h ? k0 : 0);
                const int64_t *Bhj = B + (h ? k0 : 0) * ldb + (j ? n0 : 0);
                int64_t *Tij = T + (i ? m0 : 0) * ldt + (j ? n0 : 0);
                rec_i64(cx, depth + 1, mh[i], nh[j], kh[h], Aih, lda, Bhj, ldb, Tij, ldt);
            }
    }
    if (split) {
        /* madd(C, D): C (+)= D elementwise. */
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j)
                C[i * ldc + j] = sr_add(cx->sr, C[i * ldc + j], D[i * ldd + j]);
        free(D);
        cx->temp_live -= m * n;
    }
}

/*
 * O-2 / O-3: recursive semiring product C (+)= A (x) B with base dimension b.
 * stats (may be NULL) receives {temp_total, temp_peak, leaves}.
 */
void or_rec8_i64(int sr, int64_t m, int64_t n, int64_t k,
                 const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb,
                 int64_t *C, int64_t ldc, int64_t b, uint32_t split_mask, int64_t *stats)
{
    rec_ctx cx;
    memset(&cx, 0, sizeof cx);
    cx.sr = sr;
    cx.b = b < 1 ? 1 : b;
    cx.split_mask = split_mask;
    rec_i64(&cx, 0, m, n, k, A, lda, B, ldb, C, ldc);
    if (stats) {
        stats[0] = cx.temp_total;
        stats[1] = cx.temp_peak;
        stats[2] = cx.leaves;
    }
}

/* The same recursion in double for the (+,x) semiring. */
static void rec_f64(rec_ctx *cx, int depth, int64_t m, int64_t n, int64_t k,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    double *C, int64_t ldc)
{
    if (m == 0 || n == 0 || k == 0) return;
    int64_t mx = m > n ? m : n;
    if (k > mx) mx = k;
    if (mx <= cx->b) {
        cx->leaves++;
        or_brute_f64(m, n, k, A, lda, B, ldb, C, ldc);
        return;
    }
    int64_t m0 = (m + 1) / 2, n0 = (n + 1) / 2, k0 = (k + 1) / 2;
    int64_t mh[2] = {m0, m - m0}, nh[2] = {n0, n - n0}, kh[2] = {k0, k - k0};
    int split = (cx->split_mask >> depth) & 1u;
    double *D = C;
    int64_t ldd = ldc;
    if (split) {
        D = (double *)calloc((size_t)(m * n), sizeof(double));
        ldd = n;
        cx->temp_total += m * n;
        cx->temp_live += m * n;
        if (cx->temp_live > cx->temp_peak) cx->temp_peak = cx->temp_live;
    }
    for (int h = 0; h < 2; ++h) {
        double *T = h == 0 ? C : D;
        int64_t ldt = h == 0 ? ldc : ldd;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const double *Aih = A + (i ? m0 : 0) * lda + (h ? k0 : 0);
                const double *Bhj = B + (h ? k0 : 0) * ldb + (j ? n0 : 0);
                double *Tij = T + (i ? m0 : 0) * ldt + (j ? n0 : 0);
                rec_f64(cx, depth + 1, mh[i], nh[j], kh[h], Aih, lda, Bhj, ldb, Tij, ldt);
            }
    }
    if (split) {
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) C[i * ldc + j] += D[i * ldd + j];
        free(D);
        cx->temp_live -= m * n;
    }
}

void or_rec8_f64(int64_t m, int64_t n, int64_t k,
                 const double *A, int64_t lda, const double *B, int64_t ldb,
                 double *C, int64_t ldc, int64_t b, uint32_t split_mask, int64_t *stats)
{
    rec_ctx cx;
    memset(&cx, 0, sizeof cx);
    cx.sr = OR_PLUS_TIMES;
    cx.b = b < 1 ? 1 : b;
    cx.split_mask = split_mask;
    cx.is_f64 = 1;
    rec_f64(&cx, 0, m, n, k, A, lda, B, ldb, C, ldc);
    if (stats) {
        stats[0] = cx.temp_total;
        stats[1] = cx.temp_peak;
        stats[2] = cx.leaves;
    }
}

/* --------------------------------------------------------------- Strassen */

/*
 * Strassen over a ring, written for double and for int64 through one macro
 * body (the arithmetic is the ring's + - x in both).  `variant` 0 is the
 * seven products exactly as the paper prints them; variant 1 is
 * Strassen-Winograd.  The recursion runs `depth` levels and then takes the
 * classical product.  An odd dimension is padded with one zero row/column at
 * that level, which does not change the product over a ring.
 *
 * Computes P = A B (P is overwritten; it is m x n, leading dimension n).
 */
#define DEFINE_STRASSEN(T, NAME, BASE)                                                  \
    static T *NAME##_alloc(int64_t r, int64_t c) { return (T *)calloc((size_t)(r * c), sizeof(T)); } \
    /* copy an r x c block (zero outside the source's rr x cc extent) */                \
    static void NAME##_take(T *dst, int64_t r, int64_t c, const T *src, int64_t lds,   \
                            int64_t rr, int64_t cc)                                      \
    {                                                                                    \
        for (int64_t i = 0; i < r; ++i)                                                  \
            for (int64_t j = 0; j < c; ++j)                                              \
                dst[i * c + j] = (i < rr && j < cc) ? src[i * lds + j] : (T)0;           \
    }                                                                                    \
    /* dst = x + sx*y (elementwise, all h x w, contiguous) */                            \
    static void NAME##_lin(T *dst, const T *x, int sx, const T *y, int64_t cnt)          \
    {                                                                                    \
        for (int64_t t = 0; t < cnt; ++t) dst[t] = sx > 0 ? x[t] + y[t] : x[t] - y[t];   \
    }                                                                                    \
    static void NAME##_rec(int variant, int depth, int64_t m, int64_t n, int64_t k,      \
                           const T *A, const T *B, T *P)                                 \
    {                                                                                    \
        /* A: m x k contiguous, B: k x n contiguous, P: m x n contiguous */              \
        if (depth == 0 || m < 2 || n < 2 || k < 2) {                                     \
            memset(P, 0, (size_t)(m * n) * sizeof(T));                                   \
            BASE(m, n, k, A, k, B, n, P, n);                                             \
            return;                                                                      \
        }                                                                                \
        int64_t h = (m + 1) / 2, w = (n + 1) / 2, q = (k + 1) / 2;                       \
        /* quadrants, zero padded to h x q (A), q x w (B) */                             \
        T *a[2][2], *bq[2][2];                                                           \
        for (int i = 0; i < 2; ++i)                                                      \
            for (int j = 0; j < 2; ++j) {                                                \
                a[i][j] = NAME##_alloc(h, q);                                            \
                NAME##_take(a[i][j], h, q, A + (i ? h : 0) * k + (j ? q : 0), k,         \
                            (i ? m - h : h), (j ? k - q : q));                           \
                bq[i][j] = NAME##_alloc(q, w);                                           \
                NAME##_take(bq[i][j], q, w, B + (i ? q : 0) * n + (j ? w : 0), n,        \
                            (i ? k - q : q), (j ? n - w : w));                           \
            }                                                                            \
        int64_t sa = h * q, sb = q * w, sc = h * w;                                      \
        T *S = NAME##_alloc(h, q), *Tt = NAME##_alloc(q, w);                             \
        T *Pr[8];                                                                        \
        for (int r = 1; r <= 7; ++r) Pr[r] = NAME##_alloc(h, w);                         \
        T *c[2][2];                                                                      \
        for (int i = 0; i < 2; ++i)                                                      \
            for (int j = 0; j < 2; ++j) c[i][j] = NAME##_alloc(h, w);                    \
        if (variant == 0) {                                                              \
            /* The paper's seven products (Sec. strassen). */                            \
            NAME##_lin(S, a[0][0], +1, a[1][1], sa);  /* S1 = A00 + A11 */               \
            NAME##_lin(Tt, bq[0][0], +1, bq[1][1], sb); /* T1 = B00 + B11 */             \
            NAME##_rec(variant, depth - 1, h, w, q, S, Tt, Pr[1]);                       \
            NAME##_lin(S, a[1][0], +1, a[1][1], sa);  /* S2 = A10 + A11, T2 = B00 */     \
            NAME##_rec(variant, depth - 1, h, w, q, S, bq[0][0], Pr[2]);                 \
            NAME##_lin(Tt, bq[0][1], -1, bq[1][1], sb); /* S3 = A00, T3 = B01 - B11 */   \
            NAME##_rec(variant, depth - 1, h, w, q, a[0][0], Tt, Pr[3]);                 \
            NAME##_lin(Tt, bq[1][0], -1, bq[0][0], sb); /* S4 = A11, T4 = B10 - B00 */   \
            NAME##_rec(variant, depth - 1, h, w, q, a[1][1], Tt, Pr[4]);                 \
            NAME##_lin(S, a[0][0], +1, a[0][1], sa);  /* S5 = A00 + A01, T5 = B11 */     \
            NAME##_rec(variant, depth - 1, h, w, q, S, bq[1][1], Pr[5]);                 \
            NAME##_lin(S, a[1][0], -1, a[0][0], sa);  /* S6 = A10 - A00 */               \
            NAME##_lin(Tt, bq[0][0], +1, bq[0][1], sb); /* T6 = B00 + B01 */             \
            NAME##_rec(variant, depth - 1, h, w, q, S, Tt, Pr[6]);                       \
            NAME##_lin(S, a[0][1], -1, a[1][1], sa);  /* S7 = A01 - A11 */               \
            NAME##_lin(Tt, bq[1][0], +1, bq[1][1], sb); /* T7 = B10 + B11 */             \
            NAME##_rec(variant, depth - 1, h, w, q, S, Tt, Pr[7]);                       \
            for (int64_t t = 0; t < sc; ++t) {                                           \
                c[0][0][t] = Pr[1][t] + Pr[4][t] - Pr[5][t] + Pr[7][t];                  \
                c[0][1][t] = Pr[3][t] + Pr[5][t];                                        \
                c[1][0][t] = Pr[2][t] + Pr[4][t];                                        \
                c[1][1][t] = Pr[1][t] + Pr[3][t] - Pr[2][t] + Pr[6][t];                  \
            }                                                                            \
        } else {                                                                         \
            /* Strassen-Winograd: 7 products, 8 pre-additions, 7 post-additions. */      \
            T *S1 = NAME##_alloc(h, q), *S2 = NAME##_alloc(h, q);                        \
            T *S3 = NAME##_alloc(h, q), *S4 = NAME##_alloc(h, q);                        \
            T *T1 = NAME##_alloc(q, w), *T2 = NAME##_alloc(q, w);                        \
            T *T3 = NAME##_alloc(q, w), *T4 = NAME##_alloc(q, w);                        \
            NAME##_lin(S1, a[1][0], +1, a[1][1], sa); /* S1 = A10 + A11 */               \
            NAME##_lin(S2, S1, -1, a[0][0], sa);      /* S2 = S1 - A00 */                \
            NAME##_lin(S3, a[0][0], -1, a[1][0], sa); /* S3 = A00 - A10 */               \
            NAME##_lin(S4, a[0][1], -1, S2, sa);      /* S4 = A01 - S2 */                \
            NAME##_lin(T1, bq[0][1], -1, bq[0][0], sb); /* T1 = B01 - B00 */             \
            NAME##_lin(T2, bq[1][1], -1, T1, sb);     /* T2 = B11 - T1 */                \
            NAME##_lin(T3, bq[1][1], -1, bq[0][1], sb); /* T3 = B11 - B01 */             \
            NAME##_lin(T4, T2, -1, bq[1][0], sb);     /* T4 = T2 - B10 */                \
            NAME##_rec(variant, depth - 1, h, w, q, a[0][0], bq[0][0], Pr[1]); /* M1 */  \
            NAME##_rec(variant, depth - 1, h, w, q, a[0][1], bq[1][0], Pr[2]); /* M2 */  \
            NAME##_rec(variant, depth - 1, h, w, q, S4, bq[1][1], Pr[3]);      /* M3 */  \
            NAME##_rec(variant, depth - 1, h, w, q, a[1][1], T4, Pr[4]);       /* M4 */  \
            NAME##_rec(variant, depth - 1, h, w, q, S1, T1, Pr[5]);            /* M5 */  \
            NAME##_rec(variant, depth - 1, h, w, q, S2, T2, Pr[6]);            /* M6 */  \
            NAME##_rec(variant, depth - 1, h, w, q, S3, T3, Pr[7]);            /* M7 */  \
            for (int64_t t = 0; t < sc; ++t) {                                           \
                T u1 = Pr[1][t] + Pr[6][t]; /* U1 = M1 + M6 */                           \
                T u2 = u1 + Pr[7][t];       /* U2 = U1 + M7 */                           \
                T u3 = u1 + Pr[5][t];       /* U3 = U1 + M5 */                           \
                c[0][0][t] = Pr[1][t] + Pr[2][t];                                        \
                c[0][1][t] = u3 + Pr[3][t];                                              \
                c[1][0][t] = u2 - Pr[4][t];                                              \
                c[1][1][t] = u2 + Pr[5][t];                                              \
            }                                                                            \
            free(S1); free(S2); free(S3); free(S4);                                      \
            free(T1); free(T2); free(T3); free(T4);                                      \
        }                                                                                \
        /* drop the padding while writing the quadrants back */                          \
        for (int i = 0; i < 2; ++i)                                                      \
            for (int j = 0; j < 2; ++j) {                                                \
                int64_t rr = i ? m - h : h, cc = j ? n - w : w;                          \
                for (int64_t x = 0; x < rr; ++x)                                         \
                    for (int64_t y = 0; y < cc; ++y)                                     \
                        P[((i ? h : 0) + x) * n + (j ? w : 0) + y] = c[i][j][x * w + y]; \
                free(c[i][j]);                                                           \
            }                                                                            \
        for (int r = 1; r <= 7; ++r) free(Pr[r]);                                        \
        free(S); free(Tt);                                                               \
        for (int i = 0; i < 2; ++i)                                                      \
            for (int j = 0; j < 2; ++j) { free(a[i][j]); free(bq[i][j]); }               \
    }

static void base_f64(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                     const double *B, int64_t ldb, double *C, int64_t ldc)
{
    or_brute_f64(m, n, k, A, lda, B, ldb, C, ldc);
}
static void base_i64(int64_t m, int64_t n, int64_t k, const int64_t *A, int64_t lda,
                     const int64_t *B, int64_t ldb, int64_t *C, int64_t ldc)
{
    or_brute_i64(OR_PLUS_TIMES, m, n, k, A, lda, B, ldb, C, ldc);
}

DEFINE_STRASSEN(double, strf, base_f64)
DEFINE_STRASSEN(int64_t, stri, base_i64)

/* O-4: P = A B by `depth` Strassen levels (A m x k, B k x n, P m x n; all contiguous). */
void or_strassen_f64(int variant, int depth, int64_t m, int64_t n, int64_t k,
                     const double *A, const double *B, double *P)
{
    strf_rec(variant, depth, m, n, k, A, B, P);
}

void or_strassen_i64(int variant, int depth, int64_t m, int64_t n, int64_t k,
                     const int64_t *A, const int64_t *B, int64_t *P)
{
    stri_rec(variant, depth, m, n, k, A, B, P);
}

/* ------------------------------------------------- BF16 / FP16 splitting */

/*
 * Round an IEEE binary32 value to bfloat16 (8-bit significand) with
 * round-to-nearest, ties to even, from the bit-level definition: keep the top
 * 16 bits, and add one unit in the last kept place when the dropped 16 bits
 * exceed half a unit, or equal half a unit and the kept value is odd.  NaN
 * stays NaN (quiet bit set).  Returns the 16 kept bits.
 */
uint16_t or_f32_to_bf16_rne(uint32_t bits)
{
    uint32_t exp = (bits >> 23) & 0xffu, man = bits & 0x7fffffu;
    if (exp == 0xffu && man != 0) return (uint16_t)((bits >> 16) | 0x40u);
    uint32_t kept = bits >> 16, dropped = bits & 0xffffu;
    if (dropped > 0x8000u || (dropped == 0x8000u && (kept & 1u))) kept += 1;
    return (uint16_t)kept;
}

/*
 * Round an IEEE binary32 value to binary16 (1 sign, 5 exponent bits with bias
 * 15, 10 stored significand bits) with round-to-nearest, ties to even, from
 * the bit-level definition.  The exact value is sig * 2^(e-23) with the
 * 24-bit significand sig (hidden bit included) and the unbiased exponent e.
 * A normal result (e >= -14) keeps the top 11 significand bits: drop the low
 * 13 bits and round; a carry out of the significand bumps the exponent, and
 * exponent 31 or more is infinity.  Below the normal range the result is an
 * integer multiple of 2^-24: sig is shifted right by -(e + 1) bits and
 * rounded the same way (a carry into 2^-14 gives the smallest normal, whose
 * bits follow on).  Float subnormals are far below half of 2^-24 and give
 * zero.  NaN stays NaN (quiet bit set), infinities stay infinite.
 */
uint16_t or_f32_to_fp16_rne(uint32_t bits)
{
    uint16_t sign = (uint16_t)((bits >> 16) & 0x8000u);
    uint32_t exp = (bits >> 23) & 0xffu, man = bits & 0x7fffffu;
    if (exp == 0xffu) return (uint16_t)(sign | (man ? 0x7e00u : 0x7c00u));
    if (exp == 0) return sign; /* zero or float subnormal */
    int e = (int)exp - 127;
    uint32_t sig = 0x800000u | man;
    if (e >= -14) {
        uint32_t kept = sig >> 13, dropped = sig & 0x1fffu; /* kept: 11 bits, hidden bit included */
        if (dropped > 0x1000u || (dropped == 0x1000u && (kept & 1u))) kept += 1;
        int he = e + 15;
        if (kept == 0x800u) { /* significand overflowed to 2.0 */
            kept = 0x400u;
            he += 1;
        }
        if (he >= 31) return (uint16_t)(sign | 0x7c00u);
        return (uint16_t)(sign | ((uint32_t)he << 10) | (kept & 0x3ffu));
    }
    int shift = -(e + 1); /* >= 14 */
    if (shift > 24) return sign; /* below a quarter of 2^-24 */
    uint32_t kept = sig >> shift, dropped = sig & ((1u << shift) - 1u), half = 1u << (shift - 1);
    if (dropped > half || (dropped == half && (kept & 1u))) kept += 1;
    return (uint16_t)(sign | kept);
}

/* Value of a binary16 bit pattern (exact in float64). */
double or_fp16_to_f64(uint16_t h)
{
    int sign = (h >> 15) & 1, exp = (h >> 10) & 0x1f, man = h & 0x3ff;
    double v;
    if (exp == 0)
        v = ldexp((double)man, -24);
    else if (exp == 31)
        v = man ? NAN : INFINITY;
    else
        v = ldexp((double)(0x400 | man), exp - 25);
    return sign ? -v : v;
}

/* Split each float x[i] into hi = fp16(x), lo = fp16(x - hi), both RNE. */
void or_split_fp16(int64_t cnt, const float *x, uint16_t *hi, uint16_t *lo)
{
    for (int64_t i = 0; i < cnt; ++i) {
        uint32_t b;
        memcpy(&b, &x[i], 4);
        uint16_t h = or_f32_to_fp16_rne(b);
        float r = (float)((double)x[i] - or_fp16_to_f64(h)); /* exact for |x| in the normal range */
        uint32_t rb;
        memcpy(&rb, &r, 4);
        hi[i] = h;
        lo[i] = or_f32_to_fp16_rne(rb);
    }
}

/* Split each float x[i] into hi = bf16(x), lo = bf16(x - hi), both RNE. */
void or_split_bf16(int64_t cnt, const float *x, uint16_t *hi, uint16_t *lo)
{
    for (int64_t i = 0; i < cnt; ++i) {
        uint32_t b;
        memcpy(&b, &x[i], 4);
        uint16_t h = or_f32_to_bf16_rne(b);
        uint32_t hb = (uint32_t)h << 16;
        float hf;
        memcpy(&hf, &hb, 4);
        float r = x[i] - hf; /* exact: x and hf agree in their top bits */
        uint32_t rb;
        memcpy(&rb, &r, 4);
        hi[i] = h;
        lo[i] = or_f32_to_bf16_rne(rb);
    }
}
