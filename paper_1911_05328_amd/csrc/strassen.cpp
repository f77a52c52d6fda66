// Host orchestration of mm_strassen (Sec. strassen).  Breadth-first levels
// are the straightforward parallel Strassen of Lemma par-strassen, flattened:
// all 7^depth leaf operands are formed by one pre-addition pass per operand,
// the leaf products run as one batched launch, and one post-addition pass
// adds the combined result into C.  Depth-first levels on top (SAR-Strassen,
// Lemma sar-strassen) take their seven products one after another: a round
// per digit tuple of those levels forms only its own leaves (S_r, T_r on the
// fly from A and B), multiplies them, and adds the product into the C blocks
// the round reaches at once, so the temporaries of one round are reused by
// the next.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace starmm {

namespace {

struct StrassenLayout {
    int64_t hm, hk, hn;        // leaf dims (m, k, n halved `depth` times, ceil)
    int64_t lda, ldb, ldp;     // leading dims of leaf operands / products (multiples of 4)
    int64_t sa, sb, sp;        // elements per leaf operand / product
    int64_t leaves;            // 7^(depth - df): the leaves of one round
    bool planes;               // split precision through pre-split bf16 / fp16 planes
    int64_t lpk;               // plane row length (hk rounded up to a whole staged tile, zero-filled)
    int64_t off_a, off_b, off_ap, off_bp, off_p, off_t, off_s, bytes;
};

int64_t pow7(int d) {
    int64_t r = 1;
    for (int i = 0; i < d; ++i) r *= 7;
    return r;
}

bool prec_ok(mm_precision p) {
    return p == MM_PREC_F32 || p == MM_PREC_BF16X3 || p == MM_PREC_BF16X3_HIACC || prec_fp16(p);
}

// FP16x3 scale region: |A| row maxima (m), |B| column maxima (n), then the
// leaf-row scales of A and leaf-column scales of B with their inverses
// (plane_rows entries each).
struct ScaleLayout {
    int64_t abs_a, abs_b, s_a, u_a, s_b, u_b, bytes;  // float offsets / total bytes
};
ScaleLayout scale_layout(int64_t m, int64_t n, int64_t hm, int64_t hn) {
    ScaleLayout S;
    S.abs_a = 0;
    S.abs_b = round_up(m, 64);
    S.s_a = S.abs_b + round_up(n, 64);
    S.u_a = S.s_a + plane_rows(hm);
    S.s_b = S.u_a + plane_rows(hm);
    S.u_b = S.s_b + plane_rows(hn);
    S.bytes = round_up((S.u_b + plane_rows(hn)) * 4, kAlign);
    return S;
}

// Plan of the leaf products: no banding, budget unlimited (the caller sizes it).
mm_status leaf_plan(mm_precision prec, int32_t tile, int32_t split_k, int64_t m, int64_t n, int64_t k, int64_t batch,
                    Plan* p) {
    mm_schedule s;
    std::memset(&s, 0, sizeof s);
    s.split_k = split_k <= 0 ? 1 : split_k;
    s.tile = tile;
    // Wide tiles once the batch alone fills the GPU: 256 (bf16 kernels) when
    // its tiles still cover every CU, else 128 when they cover it twice.
    if (tile == 0) {
        if (prec != MM_PREC_F32 && ceil_div(m, 256) * ceil_div(n, 256) * batch >= 256)
            s.tile = 256;
        else if (ceil_div(m, 128) * ceil_div(n, 128) * batch >= 512)
            s.tile = 128;
    }
    // the leaf products' kernel and slices; the planes (bf16 or fp16) are
    // laid out by the Strassen layout itself
    s.precision = prec == MM_PREC_F32 ? MM_PREC_F32 : MM_PREC_BF16X3;
    s.variant = MM_STRASSEN_WINOGRAD;
    s.band_rows = std::max<int64_t>(m, 1);
    s.flags = MM_FLAG_SPLIT_IN_KERNEL;
    const mm_status r = make_plan(MM_SR_PLUS_TIMES, MM_DT_F32, m, n, k, ~size_t(0) >> 1, &s, p);
    p->fp16 = prec_fp16(prec);
    return r;
}

// `df` depth-first levels on top: a round holds the 7^(depth - df) leaves
// of the breadth-first levels below them.
StrassenLayout layout(int64_t m, int64_t n, int64_t k, int depth, mm_precision prec, int32_t tile, int32_t split_k,
                      int df) {
    StrassenLayout L;
    L.hm = leaf_dim(m, depth);
    L.hk = leaf_dim(k, depth);
    L.hn = leaf_dim(n, depth);
    L.lda = round_up(std::max<int64_t>(L.hk, 1), 4);
    L.ldb = round_up(std::max<int64_t>(L.hn, 1), 4);
    L.ldp = L.ldb;
    L.sa = L.hm * L.lda;
    L.sb = L.hk * L.ldb;
    L.sp = L.hm * L.ldp;
    L.leaves = pow7(depth - df);
    L.planes = prec != MM_PREC_F32;
    L.lpk = plane_ld(L.hk);
    if (L.planes) {
        // the leaf operands as bf16 (fp16) hi/lo planes straight from the
        // pre-additions: A leaves hm x lpk, B^T leaves hn x lpk.
        L.off_a = L.off_b = 0;
        L.off_ap = 0;
        L.off_bp = round_up(L.off_ap + L.leaves * 2 * plane_rows(L.hm) * L.lpk * 2, kAlign);
        L.off_p = round_up(L.off_bp + L.leaves * 2 * plane_rows(L.hn) * L.lpk * 2, kAlign);
    } else {
        L.off_a = 0;
        L.off_b = round_up(L.off_a + L.leaves * L.sa * 4, kAlign);
        L.off_ap = L.off_bp = round_up(L.off_b + L.leaves * L.sb * 4, kAlign);
        L.off_p = L.off_ap;
    }
    L.off_t = round_up(L.off_p + L.leaves * L.sp * 4, kAlign);
    L.off_s = round_up(L.off_t + base_products_temp_bytes(prec, tile, split_k, L.hm, L.hn, L.hk, L.leaves), kAlign);
    L.bytes = L.off_s + (prec_fp16(prec) ? scale_layout(m, n, L.hm, L.hn).bytes : 0);
    return L;
}

}  // namespace

int64_t base_products_temp_bytes(mm_precision prec, int32_t tile, int32_t split_k, int64_t m, int64_t n, int64_t k,
                                 int64_t batch) {
    Plan p;
    if (leaf_plan(prec, tile, split_k, m, n, k, batch, &p) != MM_OK) return 0;
    return p.info.ws_bytes * batch;
}

hipError_t launch_base_products(mm_precision prec, int32_t tile, int32_t split_k, int64_t m, int64_t n, int64_t k,
                                const void* A, int64_t lda, int64_t stride_a, const void* B, int64_t ldb,
                                int64_t stride_b, float* C, int64_t ldc, int64_t stride_c, int64_t batch,
                                bool overwrite, float* temps, hipStream_t st, bool planes, int64_t a_plane,
                                int64_t b_plane, const float* row_unscale, const float* col_unscale) {
    Plan p;
    if (leaf_plan(prec, tile, split_k, m, n, k, batch, &p) != MM_OK) return hipErrorInvalidValue;
    SliceArgs sa;
    sa.batch = (int32_t)batch;
    sa.stride_a = stride_a;
    sa.stride_b = stride_b;
    sa.stride_c = stride_c;
    sa.overwrite = overwrite ? 1 : 0;
    sa.temp_batch_stride = p.info.temp_elems;
    sa.a_plane = a_plane;
    sa.b_plane = b_plane;
    sa.row_unscale = row_unscale;
    sa.col_unscale = col_unscale;
    hipError_t e;
    if (p.family == KF_F32_MFMA)
        e = launch_f32_tiles(p, m, n, k, (const float*)A, lda, (const float*)B, ldb, C, ldc, temps, 0, m, sa, st);
    else
        e = launch_bf16_tiles(p, planes ? (p.fp16 ? 4 : 2) : 0, m, n, k, A, lda, B, ldb, C, ldc, temps, 0, m, sa, st);
    if (e == hipSuccess && p.info.sar_levels > 0)
        e = launch_merge_f32(p, C, ldc, temps, 0, m, n, st, batch, stride_c, p.info.temp_elems);
    return e;
}

namespace {

// Depth 0 in split precision: both operands split once into k-tiled bf16
// (fp16) hi/lo planes (B transposed) ahead of the product's temporaries.
int64_t depth0_plane_ld(int64_t k) { return plane_ld(k); }
int64_t depth0_planes_bytes(int64_t m, int64_t n, int64_t k, mm_precision prec) {
    if (prec == MM_PREC_F32) return 0;
    return round_up((plane_rows(m) + plane_rows(n)) * depth0_plane_ld(k) * 4, kAlign);
}

// Growth bound of the pre-additions: a leaf entry is a signed sum of at
// most 2^depth (classic) or 4^depth (Winograd) source entries.
float preadd_growth(int depth, mm_strassen_variant variant) {
    return (float)(int64_t(1) << ((variant == MM_STRASSEN_WINOGRAD ? 2 : 1) * depth));
}

// FP16x3 scales (one power of two per leaf row of A and per leaf column of
// B) from the operands' row / column maxima.
hipError_t fp16_scales(const float* A, int64_t lda, const float* B, int64_t ldb, int64_t m, int64_t n, int64_t k,
                       int depth, mm_strassen_variant variant, int64_t hm, int64_t hn, float* S,
                       const ScaleLayout& L, hipStream_t st) {
    const float g = preadd_growth(depth, variant);
    hipError_t e = launch_absmax_rows(A, lda, m, k, S + L.abs_a, st);
    if (e == hipSuccess) e = launch_absmax_cols(B, ldb, k, n, S + L.abs_b, st);
    if (e == hipSuccess) e = launch_pow2_scales(S + L.abs_a, make_paths(m, depth), depth, g, hm, S + L.s_a, S + L.u_a, st);
    if (e == hipSuccess) e = launch_pow2_scales(S + L.abs_b, make_paths(n, depth), depth, g, hn, S + L.s_b, S + L.u_b, st);
    return e;
}

}  // namespace

int64_t strassen_ws_bytes(int64_t m, int64_t n, int64_t k, int32_t depth, mm_precision prec, int32_t tile,
                          int32_t split_k, int32_t df) {
    if (m <= 0 || n <= 0 || k <= 0) return 0;  // an empty product launches nothing
    if (depth == 0)
        return depth0_planes_bytes(m, n, k, prec) +
               (prec_fp16(prec) ? round_up(base_products_temp_bytes(prec, tile, split_k, m, n, k, 1), kAlign) +
                                      scale_layout(m, n, m, n).bytes
                                : base_products_temp_bytes(prec, tile, split_k, m, n, k, 1));
    return layout(m, n, k, depth, prec, tile, split_k, df).bytes;
}

int32_t strassen_choose_df(int64_t m, int64_t n, int64_t k, int32_t top, int32_t depth, mm_precision prec,
                           int32_t tile, int32_t split_k, size_t budget) {
    for (int32_t df = 0; df <= depth; ++df)
        if (star_strassen_ws_bytes(m, n, k, top, depth, prec, tile, split_k, df) <= (int64_t)budget) return df;
    return -1;
}

mm_status strassen_run(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B, int64_t ldb,
                       float* C, int64_t ldc, int32_t depth, mm_strassen_variant variant, mm_precision prec,
                       int32_t tile, int32_t split_k, int32_t df, void* workspace, size_t workspace_bytes,
                       hipStream_t st) {
    if (m < 0 || n < 0 || k < 0) return MM_ERR_INVALID_ARG;
    if (depth < 0 || depth > kMaxStrassenDepth) return MM_ERR_INVALID_ARG;
    if (df < 0 || df > depth) return MM_ERR_INVALID_ARG;
    if (variant != MM_STRASSEN_CLASSIC && variant != MM_STRASSEN_WINOGRAD) return MM_ERR_INVALID_ARG;
    if (!prec_ok(prec)) return MM_ERR_INVALID_ARG;
    if (tile != 0 && tile != 32 && tile != 64 && tile != 128 && tile != 256) return MM_ERR_INVALID_ARG;
    if (split_k < 0 || split_k > kMaxSplit || (split_k > 0 && !is_pow2(split_k))) return MM_ERR_INVALID_ARG;
    if (lda < (k > 1 ? k : 1) || ldb < (n > 1 ? n : 1) || ldc < (n > 1 ? n : 1)) return MM_ERR_INVALID_ARG;
    if ((m > 0 && k > 0 && !A) || (k > 0 && n > 0 && !B) || (m > 0 && n > 0 && !C)) return MM_ERR_INVALID_ARG;
    if (!workspace_ok(workspace, workspace_bytes)) return MM_ERR_INVALID_ARG;
    const int64_t kDimMax = int64_t(1) << 31;
    if (m > kDimMax || n > kDimMax || k > kDimMax) return MM_ERR_INVALID_ARG;
    const int64_t need = strassen_ws_bytes(m, n, k, depth, prec, tile, split_k, df);
    if ((int64_t)workspace_bytes < need) return MM_ERR_WORKSPACE;
    if (m == 0 || n == 0 || k == 0) return MM_OK;
    hipError_t e;
    if (depth == 0 && prec == MM_PREC_F32) {
        e = launch_base_products(prec, tile, split_k, m, n, k, A, lda, 0, B, ldb, 0, C, ldc, 0, 1, false,
                                 static_cast<float*>(workspace), st);
    } else if (depth == 0) {
        const int64_t ldp = depth0_plane_ld(k);
        const int64_t a_plane = plane_rows(m) * ldp, b_plane = plane_rows(n) * ldp;
        uint16_t* Ap = static_cast<uint16_t*>(workspace);
        uint16_t* Bp = Ap + 2 * a_plane;
        const int64_t pb = depth0_planes_bytes(m, n, k, prec);
        float* T = reinterpret_cast<float*>(static_cast<char*>(workspace) + pb);
        const float *sa = nullptr, *ua = nullptr, *sb = nullptr, *ub = nullptr;
        e = hipSuccess;
        if (prec_fp16(prec)) {
            const ScaleLayout SL = scale_layout(m, n, m, n);
            float* S = reinterpret_cast<float*>(
                static_cast<char*>(workspace) + pb +
                round_up(base_products_temp_bytes(prec, tile, split_k, m, n, k, 1), kAlign));
            e = fp16_scales(A, lda, B, ldb, m, n, k, 0, variant, m, n, S, SL, st);
            sa = S + SL.s_a, ua = S + SL.u_a, sb = S + SL.s_b, ub = S + SL.u_b;
        }
        if (e == hipSuccess) e = launch_split_rows(A, lda, 0, m, k, Ap, ldp, 0, a_plane, 1, st, sa);
        if (e == hipSuccess) e = launch_split_transpose(B, ldb, 0, k, n, Bp, ldp, 0, b_plane, 1, st, sb);
        if (e == hipSuccess)
            e = launch_base_products(prec, tile, split_k, m, n, k, Ap, ldp, 0, Bp, ldp, 0, C, ldc, 0, 1, false, T, st,
                                     true, a_plane, b_plane, ua, ub);
    } else {
        const StrassenLayout L = layout(m, n, k, depth, prec, tile, split_k, df);
        char* ws = static_cast<char*>(workspace);
        float* SA = reinterpret_cast<float*>(ws + L.off_a);
        float* SB = reinterpret_cast<float*>(ws + L.off_b);
        float* P = reinterpret_cast<float*>(ws + L.off_p);
        float* T = reinterpret_cast<float*>(ws + L.off_t);
        const bool f64 = prec_hiacc(prec);
        const PathTable rm = make_paths(m, depth), rk = make_paths(k, depth), rn = make_paths(n, depth);
        uint16_t* Ap = reinterpret_cast<uint16_t*>(ws + L.off_ap);
        uint16_t* Bp = reinterpret_cast<uint16_t*>(ws + L.off_bp);
        const int64_t a_plane = plane_rows(L.hm) * L.lpk, b_plane = plane_rows(L.hn) * L.lpk;
        const float *sa = nullptr, *ua = nullptr, *sb = nullptr, *ub = nullptr;
        e = hipSuccess;
        if (L.planes && prec_fp16(prec)) {
            // one scale per leaf row / column, whatever the round
            const ScaleLayout SL = scale_layout(m, n, L.hm, L.hn);
            float* S = reinterpret_cast<float*>(ws + L.off_s);
            e = fp16_scales(A, lda, B, ldb, m, n, k, depth, variant, L.hm, L.hn, S, SL, st);
            sa = S + SL.s_a, ua = S + SL.u_a, sb = S + SL.s_b, ub = S + SL.u_b;
        }
        // rounds: digit tuples of the depth-first levels in ascending order
        // (level 0 most significant), so the float result is deterministic
        const int bf = depth - df;
        const int64_t rounds = pow7(df);
        for (int64_t round = 0; round < rounds && e == hipSuccess; ++round) {
            uint32_t fix = kAllFree;
            int digit[kMaxStrassenDepth] = {};
            for (int l = df - 1, q = (int)round; l >= 0; --l, q /= 7) {
                digit[l] = q % 7;
                fix = (fix & ~(7u << (3 * l))) | ((uint32_t)digit[l] << (3 * l));
            }
            if (L.planes) {
                // both operands' leaves straight to k-tiled bf16 (fp16) hi/lo
                // planes (B read in place for the B^T leaves)
                e = launch_strassen_pre_planes(depth, variant, f64, 0, A, lda, rm, rk, Ap, L.hm, L.lpk, 2 * a_plane,
                                               a_plane, st, sa, fix);
                if (e == hipSuccess)
                    e = launch_strassen_pre_planes(depth, variant, f64, 2, B, ldb, rn, rk, Bp, L.hn, L.lpk,
                                                   2 * b_plane, b_plane, st, sb, fix);
                if (e == hipSuccess)
                    e = launch_base_products(prec, tile, split_k, L.hm, L.hn, L.hk, Ap, L.lpk, 2 * a_plane, Bp, L.lpk,
                                             2 * b_plane, P, L.ldp, L.sp, L.leaves, true, T, st, true, a_plane,
                                             b_plane, ua, ub);
            } else {
                e = launch_strassen_pre(depth, variant, f64, 0, A, lda, rm, rk, SA, L.hm, L.hk, L.lda, L.sa, st, fix);
                if (e == hipSuccess)
                    e = launch_strassen_pre(depth, variant, f64, 1, B, ldb, rk, rn, SB, L.hk, L.hn, L.ldb, L.sb, st,
                                            fix);
                if (e == hipSuccess)
                    e = launch_base_products(prec, tile, split_k, L.hm, L.hn, L.hk, SA, L.lda, L.sa, SB, L.ldb, L.sb,
                                             P, L.ldp, L.sp, L.leaves, true, T, st);
            }
            if (e != hipSuccess) break;
            if (df == 0) {
                e = launch_strassen_post(depth, variant, f64, P, L.ldp, L.sp, rm, rn, C, ldc, L.hm, L.hn, st);
            } else {
                // the C blocks of the depth-first grid this round reaches:
                // block (I, J) takes gamma(r_0; i_0, j_0) ... gamma(r_{df-1};
                // i_{df-1}, j_{df-1}) times the round's product
                RoundTargets tg;
                tg.count = 0;
                for (int I = 0; I < (1 << df); ++I)
                    for (int J = 0; J < (1 << df); ++J) {
                        int g = 1;
                        for (int l = 0; l < df && g != 0; ++l)
                            g *= strassen_gamma(variant, digit[l], (I >> (df - 1 - l)) & 1, (J >> (df - 1 - l)) & 1);
                        if (g != 0) tg.target[tg.count++] = I | (J << 8) | ((g < 0 ? 1 : 0) << 16);
                    }
                e = launch_strassen_post_round(bf, variant, f64, P, L.ldp, L.sp, rm, rn, C, ldc, L.hm, L.hn, tg, st);
            }
        }
    }
    if (e != hipSuccess) {
        set_last_error(std::string("mm_strassen launch: ") + hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    return MM_OK;
}

int64_t star_strassen_ws_bytes(int64_t m, int64_t n, int64_t k, int32_t top, int32_t depth, mm_precision prec,
                               int32_t tile, int32_t split_k, int32_t df) {
    // the largest sub-product is the first one (ceil halves)
    return strassen_ws_bytes(leaf_dim(m, top), leaf_dim(n, top), leaf_dim(k, top), depth, prec, tile, split_k, df);
}

mm_status star_strassen_run(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B,
                            int64_t ldb, float* C, int64_t ldc, int32_t top, int32_t depth,
                            mm_strassen_variant variant, mm_precision prec, int32_t tile, int32_t split_k,
                            int32_t df, void* workspace, size_t workspace_bytes, hipStream_t st) {
    if (top == 0)
        return strassen_run(m, n, k, A, lda, B, ldb, C, ldc, depth, variant, prec, tile, split_k, df, workspace,
                            workspace_bytes, st);
    if (top < 0 || top > kMaxStarStrassen || m < 0 || n < 0 || k < 0) return MM_ERR_INVALID_ARG;
    if (lda < (k > 1 ? k : 1) || ldb < (n > 1 ? n : 1) || ldc < (n > 1 ? n : 1)) return MM_ERR_INVALID_ARG;
    if ((m > 0 && k > 0 && !A) || (k > 0 && n > 0 && !B) || (m > 0 && n > 0 && !C)) return MM_ERR_INVALID_ARG;
    if ((int64_t)workspace_bytes < star_strassen_ws_bytes(m, n, k, top, depth, prec, tile, split_k, df))
        return MM_ERR_WORKSPACE;
    if (m == 0 || n == 0 || k == 0) return MM_OK;
    // The top levels of the 8-way recursion: C block (I, J) accumulates the
    // products of A's row block I and B's column block J over the k-slices L
    // in ascending order, so the float result does not depend on timing.
    const PathTable rm = make_paths(m, top), rn = make_paths(n, top), rk = make_paths(k, top);
    const int nb = 1 << top;
    for (int q = 0; q < nb * nb; ++q) {
        // C blocks in the recursion's quadrant order (bits of I and J interleaved)
        int I = 0, J = 0;
        for (int b = 0; b < top; ++b) {
            I |= ((q >> (2 * b + 1)) & 1) << b;
            J |= ((q >> (2 * b)) & 1) << b;
        }
        if (rm.ext[I] == 0 || rn.ext[J] == 0) continue;
        for (int L = 0; L < nb; ++L) {
            if (rk.ext[L] == 0) continue;
            const mm_status s = strassen_run(rm.ext[I], rn.ext[J], rk.ext[L], A + rm.off[I] * lda + rk.off[L], lda,
                                             B + rk.off[L] * ldb + rn.off[J], ldb, C + rm.off[I] * ldc + rn.off[J],
                                             ldc, depth, variant, prec, tile, split_k, df, workspace,
                                             workspace_bytes, st);
            if (s != MM_OK) return s;
        }
    }
    return MM_OK;
}

}  // namespace starmm

using namespace starmm;

extern "C" {

size_t mm_strassen_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t depth, mm_strassen_variant variant,
                                   mm_precision prec) {
    if (m < 0 || n < 0 || k < 0 || depth < 0 || depth > kMaxStrassenDepth) return 0;
    if (variant != MM_STRASSEN_CLASSIC && variant != MM_STRASSEN_WINOGRAD) return 0;
    if (!prec_ok(prec)) return 0;
    return (size_t)strassen_ws_bytes(m, n, k, depth, prec, 0, 1, 0);
}

mm_status mm_strassen_coefficients(mm_strassen_variant variant, int8_t* alpha, int8_t* beta, int8_t* gamma) {
    if (variant != MM_STRASSEN_CLASSIC && variant != MM_STRASSEN_WINOGRAD) return MM_ERR_INVALID_ARG;
    if (!alpha || !beta || !gamma) return MM_ERR_INVALID_ARG;
    for (int r = 0; r < 7; ++r)
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                alpha[r * 4 + i * 2 + j] = (int8_t)strassen_alpha(variant, r, i, j);
                beta[r * 4 + i * 2 + j] = (int8_t)strassen_beta(variant, r, i, j);
                gamma[r * 4 + i * 2 + j] = (int8_t)strassen_gamma(variant, r, i, j);
            }
    return MM_OK;
}

mm_status mm_strassen(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B, int64_t ldb,
                      float* C, int64_t ldc, int32_t depth, mm_strassen_variant variant, mm_precision prec,
                      void* workspace, size_t workspace_bytes, void* stream) {
    // every level breadth-first when the workspace holds it, else the fewest
    // depth-first levels on top that fit (MM_ERR_WORKSPACE if none does)
    int32_t df = 0;
    if (depth >= 0 && depth <= kMaxStrassenDepth && prec_ok(prec) && m >= 0 && n >= 0 && k >= 0) {
        df = strassen_choose_df(m, n, k, 0, depth, prec, 0, 1, workspace_bytes);
        if (df < 0) return MM_ERR_WORKSPACE;
    }
    return strassen_run(m, n, k, A, lda, B, ldb, C, ldc, depth, variant, prec, 0, 1, df, workspace, workspace_bytes,
                        (hipStream_t)stream);
}

}  // extern "C"
