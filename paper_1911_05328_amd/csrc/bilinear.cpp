// General bilinear level (eq. bilinear, closing remarks of Sec. strassen):
// scheme builders and checks (host only) and the orchestration of one level
// above the BF16x3 base product: pre-additions into planes, the batched
// products, the post-addition into C.
#include <cstring>

#include "bilinear.hpp"
#include "internal.hpp"

namespace starmm {

namespace {

bool shape_ok(const mm_bilinear_scheme* s) {
    return s && s->g >= 1 && s->g <= MM_BILINEAR_MAX_GRID && s->products >= 1 &&
           s->products <= MM_BILINEAR_MAX_PRODUCTS;
}

// sum_r alpha[r,(i,l)] beta[r,(l',j)] gamma[(i',j'),r] against the matrix
// multiplication tensor, for every index
bool reproduces_mm(const mm_bilinear_scheme* s) {
    const int g = s->g, R = s->products, gg = g * g;
    for (int i = 0; i < g; ++i)
        for (int l = 0; l < g; ++l)
            for (int l2 = 0; l2 < g; ++l2)
                for (int j = 0; j < g; ++j)
                    for (int i2 = 0; i2 < g; ++i2)
                        for (int j2 = 0; j2 < g; ++j2) {
                            int64_t t = 0;
                            for (int r = 0; r < R; ++r)
                                t += (int64_t)s->alpha[r * gg + i * g + l] * s->beta[r * gg + l2 * g + j] *
                                     s->gamma[(i2 * g + j2) * R + r];
                            if (t != ((i == i2 && l == l2 && j == j2) ? 1 : 0)) return false;
                        }
    return true;
}

BlockTable blocks(int64_t dim, int g) {
    BlockTable t{};
    const int64_t h = ceil_div(dim, g);
    for (int i = 0; i < g; ++i) {
        t.off[i] = i * h;
        t.ext[i] = std::max<int64_t>(0, std::min<int64_t>(h, dim - i * h));
    }
    return t;
}

struct BilinearLayout {
    int64_t hm, hk, hn, lpk, ldp, sp, a_plane, b_plane;
    int64_t off_ap, off_bp, off_p, off_t, bytes;
};

BilinearLayout layout(int64_t m, int64_t n, int64_t k, int g, int R) {
    BilinearLayout L;
    L.hm = ceil_div(m, g);
    L.hk = ceil_div(k, g);
    L.hn = ceil_div(n, g);
    L.lpk = plane_ld(L.hk);
    L.ldp = round_up(std::max<int64_t>(L.hn, 1), 4);
    L.sp = L.hm * L.ldp;
    L.a_plane = plane_rows(L.hm) * L.lpk;
    L.b_plane = plane_rows(L.hn) * L.lpk;
    L.off_ap = 0;
    L.off_bp = round_up(L.off_ap + R * 2 * L.a_plane * 2, kAlign);
    L.off_p = round_up(L.off_bp + R * 2 * L.b_plane * 2, kAlign);
    L.off_t = round_up(L.off_p + R * L.sp * 4, kAlign);
    L.bytes = L.off_t + base_products_temp_bytes(MM_PREC_BF16X3, 0, 1, L.hm, L.hn, L.hk, R);
    return L;
}

}  // namespace

}  // namespace starmm

using namespace starmm;

extern "C" {

mm_status mm_bilinear_builtin(mm_bilinear_kind kind, int32_t param, mm_bilinear_scheme* out) {
    if (!out) return MM_ERR_INVALID_ARG;
    mm_bilinear_scheme s;
    std::memset(&s, 0, sizeof s);
    if (kind == MM_BILINEAR_CLASSICAL) {
        const int g = param;
        if (g < 1 || g > MM_BILINEAR_MAX_GRID || g * g * g > MM_BILINEAR_MAX_PRODUCTS) return MM_ERR_INVALID_ARG;
        s.g = g;
        s.products = g * g * g;
        int r = 0;
        for (int i = 0; i < g; ++i)
            for (int l = 0; l < g; ++l)
                for (int j = 0; j < g; ++j, ++r) {
                    s.alpha[r * g * g + i * g + l] = 1;
                    s.beta[r * g * g + l * g + j] = 1;
                    s.gamma[(i * g + j) * s.products + r] = 1;
                }
    } else if (kind == MM_BILINEAR_STRASSEN) {
        int8_t a[28], b[28], c[28];
        if (mm_strassen_coefficients((mm_strassen_variant)param, a, b, c) != MM_OK) return MM_ERR_INVALID_ARG;
        s.g = 2;
        s.products = 7;
        for (int r = 0; r < 7; ++r)
            for (int q = 0; q < 4; ++q) {
                s.alpha[r * 4 + q] = a[r * 4 + q];
                s.beta[r * 4 + q] = b[r * 4 + q];
                s.gamma[q * 7 + r] = c[r * 4 + q];
            }
    } else {
        return MM_ERR_INVALID_ARG;
    }
    *out = s;
    return MM_OK;
}

mm_status mm_bilinear_product(const mm_bilinear_scheme* s1, const mm_bilinear_scheme* s2, mm_bilinear_scheme* out) {
    if (!shape_ok(s1) || !shape_ok(s2) || !out) return MM_ERR_INVALID_ARG;
    const int g1 = s1->g, g2 = s2->g, g = g1 * g2, R1 = s1->products, R2 = s2->products;
    if (g > MM_BILINEAR_MAX_GRID || R1 * R2 > MM_BILINEAR_MAX_PRODUCTS) return MM_ERR_INVALID_ARG;
    mm_bilinear_scheme s;
    std::memset(&s, 0, sizeof s);
    s.g = g;
    s.products = R1 * R2;
    // fine block of fine index (a2, b2) inside coarse block (a1, b1)
    auto fine = [&](int b1, int b2) {
        const int i1 = b1 / g1, l1 = b1 % g1, i2 = b2 / g2, l2 = b2 % g2;
        return (i1 * g2 + i2) * g + (l1 * g2 + l2);
    };
    for (int r1 = 0; r1 < R1; ++r1)
        for (int r2 = 0; r2 < R2; ++r2) {
            const int r = r1 * R2 + r2;
            for (int b1 = 0; b1 < g1 * g1; ++b1)
                for (int b2 = 0; b2 < g2 * g2; ++b2) {
                    const int f = fine(b1, b2);
                    const int a = s1->alpha[r1 * g1 * g1 + b1] * s2->alpha[r2 * g2 * g2 + b2];
                    const int b = s1->beta[r1 * g1 * g1 + b1] * s2->beta[r2 * g2 * g2 + b2];
                    const int c = s1->gamma[b1 * R1 + r1] * s2->gamma[b2 * R2 + r2];
                    if (a < -128 || a > 127 || b < -128 || b > 127 || c < -128 || c > 127) return MM_ERR_INVALID_ARG;
                    s.alpha[r * g * g + f] = (int8_t)a;
                    s.beta[r * g * g + f] = (int8_t)b;
                    s.gamma[f * s.products + r] = (int8_t)c;
                }
        }
    *out = s;
    return MM_OK;
}

mm_status mm_bilinear_scheme_check(const mm_bilinear_scheme* s) {
    return shape_ok(s) && reproduces_mm(s) ? MM_OK : MM_ERR_INVALID_ARG;
}

size_t mm_bilinear_workspace_bytes(int64_t m, int64_t n, int64_t k, const mm_bilinear_scheme* s, mm_precision prec) {
    if (!shape_ok(s) || prec != MM_PREC_BF16X3 || m < 0 || n < 0 || k < 0) return 0;
    if (m == 0 || n == 0 || k == 0) return 0;
    return (size_t)layout(m, n, k, s->g, s->products).bytes;
}

mm_status mm_bilinear(int64_t m, int64_t n, int64_t k, const float* A, int64_t lda, const float* B, int64_t ldb,
                      float* C, int64_t ldc, const mm_bilinear_scheme* s, mm_precision prec, void* workspace,
                      size_t workspace_bytes, void* stream) {
    if (m < 0 || n < 0 || k < 0) return MM_ERR_INVALID_ARG;
    if (lda < (k > 1 ? k : 1) || ldb < (n > 1 ? n : 1) || ldc < (n > 1 ? n : 1)) return MM_ERR_INVALID_ARG;
    if ((m > 0 && k > 0 && !A) || (k > 0 && n > 0 && !B) || (m > 0 && n > 0 && !C)) return MM_ERR_INVALID_ARG;
    if (!workspace_ok(workspace, workspace_bytes)) return MM_ERR_INVALID_ARG;
    const int64_t kDimMax = int64_t(1) << 31;
    if (m > kDimMax || n > kDimMax || k > kDimMax) return MM_ERR_INVALID_ARG;
    if (mm_bilinear_scheme_check(s) != MM_OK) return MM_ERR_INVALID_ARG;
    if (prec != MM_PREC_BF16X3) return MM_ERR_UNSUPPORTED;
    if (m == 0 || n == 0 || k == 0) return MM_OK;
    const int g = s->g, R = s->products;
    const BilinearLayout L = layout(m, n, k, g, R);
    if ((int64_t)workspace_bytes < L.bytes) return MM_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char* ws = static_cast<char*>(workspace);
    uint16_t* Ap = reinterpret_cast<uint16_t*>(ws + L.off_ap);
    uint16_t* Bp = reinterpret_cast<uint16_t*>(ws + L.off_bp);
    float* P = reinterpret_cast<float*>(ws + L.off_p);
    float* T = reinterpret_cast<float*>(ws + L.off_t);
    const BlockTable rm = blocks(m, g), rk = blocks(k, g), rn = blocks(n, g);
    BilinearSide sa{}, sb{};
    BilinearOut so{};
    sa.products = sb.products = so.products = R;
    std::memcpy(sa.coef, s->alpha, (size_t)R * g * g);
    std::memcpy(sb.coef, s->beta, (size_t)R * g * g);
    std::memcpy(so.coef, s->gamma, (size_t)g * g * R);
    hipError_t e = launch_bilinear_pre(g, false, A, lda, rm, rk, Ap, plane_rows(L.hm), L.lpk, 2 * L.a_plane,
                                       L.a_plane, sa, st);
    if (e == hipSuccess)
        e = launch_bilinear_pre(g, true, B, ldb, rn, rk, Bp, plane_rows(L.hn), L.lpk, 2 * L.b_plane, L.b_plane, sb,
                                st);
    if (e == hipSuccess)
        e = launch_base_products(MM_PREC_BF16X3, 0, 1, L.hm, L.hn, L.hk, Ap, L.lpk, 2 * L.a_plane, Bp, L.lpk,
                                 2 * L.b_plane, P, L.ldp, L.sp, R, true, T, st, true, L.a_plane, L.b_plane, nullptr,
                                 nullptr);
    if (e == hipSuccess) e = launch_bilinear_post(g, P, L.ldp, L.sp, rm, rn, C, ldc, L.hm, L.hn, so, st);
    if (e != hipSuccess) {
        set_last_error(std::string("mm_bilinear launch: ") + hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    return MM_OK;
}

}  // extern "C"
