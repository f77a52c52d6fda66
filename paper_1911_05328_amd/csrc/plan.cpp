// Host planner: resolves a schedule for one product and carves the caller's
// workspace.  Pure host code (no HIP calls), so it is exercised by the CPU
// tests through mm_plan().
//
// The schedule is the GPU reading of the paper's recursion (Sec. mm):
//  * the 8-way recursion of eq. (mm-dac) is flattened: every base-case
//    output tile is one workgroup, visited in the recursion's quadrant
//    order;
//  * the top log2(s) levels split k into halves that run concurrently.  At
//    TAR levels (Sec. tar-mm) both halves update C and the writes are
//    serialised by atomic (+); at SAR/CO3 levels (Fig. mm-n3, Sec. sar-mm)
//    the k-half-0 product keeps the parent's storage (lazy allocation) and
//    the k-half-1 product gets a temporary, merged by madd.  TAR above
//    depth star_depth and SAR below is the STAR hybrid (Sec. star-mm);
//  * the temporaries of one band of C rows are reused by the next band, so
//    the live temporary space is bounded by what runs concurrently, not by
//    the problem (the allocator-reuse argument of Sec. sar-mm).
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace starmm {

namespace {

constexpr int64_t kCUs = 256;

bool valid_tile(int t) { return t == 32 || t == 64 || t == 128; }

// The bf16 MFMA kernels also have a 256 x 256 tile (4 waves of 128 x 128).
bool valid_tile_for(KernelFamily f, int t) {
    return valid_tile(t) || (t == 256 && (f == KF_BF16X3_MFMA || f == KF_BF16_MFMA || f == KF_F16_MFMA));
}

int tile_k_for(KernelFamily f) {
    switch (f) {
        case KF_SEMIRING_I32: return 16;
        case KF_F32_MFMA: return 16;
        default: return 32;
    }
}

int default_tile(int64_t m, int64_t n) {
    auto tiles = [&](int64_t t) { return ceil_div(m, t) * ceil_div(n, t); };
    if (m >= 128 && n >= 128 && tiles(128) >= 2 * kCUs) return 128;
    if (m >= 64 && n >= 64 && tiles(64) >= kCUs / 2) return 64;
    if (m >= 128 && n >= 128) return 128;
    return m >= 64 && n >= 64 ? 64 : 32;
}

}  // namespace

mm_status make_plan(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                    size_t workspace_bytes, const mm_schedule* sched, Plan* plan) {
    if (!plan) return MM_ERR_INVALID_ARG;
    std::memset(plan, 0, sizeof(*plan));
    if (m < 0 || n < 0 || k < 0) return MM_ERR_INVALID_ARG;
    if (sr != MM_SR_PLUS_TIMES && sr != MM_SR_MIN_PLUS && sr != MM_SR_MAX_PLUS && sr != MM_SR_MAX_MIN &&
        sr != MM_SR_OR_AND)
        return MM_ERR_INVALID_ARG;
    if (dt != MM_DT_I32 && dt != MM_DT_F32 && dt != MM_DT_BF16 && dt != MM_DT_F16) return MM_ERR_INVALID_ARG;
    // Sizes far beyond one GPU's memory are rejected so that index arithmetic
    // in int64 never overflows.
    const int64_t kDimMax = int64_t(1) << 31;
    if (m > kDimMax || n > kDimMax || k > kDimMax) return MM_ERR_INVALID_ARG;

    mm_schedule s;
    std::memset(&s, 0, sizeof s);
    if (sched) s = *sched;
    if (s.split_k < 0 || s.star_depth < 0 || s.strassen_depth < 0 || s.band_rows < 0 ||
        s.tile < 0)
        return MM_ERR_INVALID_ARG;
    if (s.variant != MM_STRASSEN_CLASSIC && s.variant != MM_STRASSEN_WINOGRAD)
        return MM_ERR_INVALID_ARG;
    if (s.flags & ~(MM_FLAG_NONDETERMINISTIC | MM_FLAG_SPLIT_IN_KERNEL | MM_FLAG_PERSISTENT | MM_FLAG_CHECKED_RANGE))
        return MM_ERR_INVALID_ARG;
    if ((s.flags & MM_FLAG_CHECKED_RANGE) && (sr == MM_SR_PLUS_TIMES || sr == MM_SR_OR_AND))
        return MM_ERR_INVALID_ARG;

    // Semiring / dtype / precision combinations.
    KernelFamily fam;
    if (sr != MM_SR_PLUS_TIMES) {
        if (dt != MM_DT_I32) return MM_ERR_UNSUPPORTED;
        // Strassen needs the inverse of (+) (Sec. strassen): not a ring.
        if (s.strassen_depth > 0) return MM_ERR_UNSUPPORTED;
        if (s.precision != 0) return MM_ERR_INVALID_ARG;
        fam = KF_SEMIRING_I32;
    } else {
        if (dt == MM_DT_I32) return MM_ERR_UNSUPPORTED;
        if (s.strassen_depth > kMaxStrassenDepth) return MM_ERR_INVALID_ARG;
        if (dt == MM_DT_BF16) {
            if (s.precision != MM_PREC_F32 && s.precision != MM_PREC_BF16) return MM_ERR_INVALID_ARG;
            s.precision = MM_PREC_BF16;
            fam = KF_BF16_MFMA;
        } else if (dt == MM_DT_F16) {
            // fp16 inputs: one fp16 product, fp32 accumulation
            if (s.precision != MM_PREC_F32) return MM_ERR_INVALID_ARG;
            fam = KF_F16_MFMA;
        } else {
            switch (s.precision) {
                case MM_PREC_F32: fam = KF_F32_MFMA; break;
                case MM_PREC_BF16X3:
                case MM_PREC_BF16X3_HIACC:
                case MM_PREC_FP16X3:
                case MM_PREC_FP16X3_HIACC: fam = KF_BF16X3_MFMA; break;
                default: return MM_ERR_INVALID_ARG;
            }
        }
        // Strassen levels through mm_semiring are served by mm_strassen's path.
        if (s.strassen_depth > 0 && dt != MM_DT_F32) return MM_ERR_UNSUPPORTED;
    }
    const bool exact = fam == KF_SEMIRING_I32;
    if ((s.flags & MM_FLAG_PERSISTENT) && !exact) return MM_ERR_UNSUPPORTED;
    // An empty product (C unchanged for k = 0, nothing at all for m = 0 or
    // n = 0) launches nothing, so it needs no workspace whatever the schedule.
    const bool empty = m == 0 || n == 0 || k == 0;

    // FP16x3 (scaled operands, pre-split planes) runs through the same
    // orchestration as the Strassen levels, depth 0 included.
    if (s.strassen_depth > 0 || prec_fp16(s.precision)) {
        if (prec_fp16(s.precision) && (s.flags & MM_FLAG_SPLIT_IN_KERNEL)) return MM_ERR_INVALID_ARG;
        // Strassen levels above the base product (Sec. strassen): the schedule's
        // tile and split_k apply to the 7^depth leaf products.
        if (s.tile != 0 && !valid_tile_for(fam, s.tile)) return MM_ERR_INVALID_ARG;
        if (s.split_k == 0) s.split_k = 1;
        if (!is_pow2(s.split_k) || s.split_k > kMaxSplit) return MM_ERR_INVALID_ARG;
        if (s.band_rows != 0) return MM_ERR_INVALID_ARG;
        // star_depth: 8-way levels above the Strassen levels (STAR-Strassen)
        if (s.star_depth > kMaxStarStrassen) return MM_ERR_INVALID_ARG;
        const mm_precision prec = (mm_precision)s.precision;
        // depth-first levels (SAR-Strassen) on top of breadth-first ones: the
        // planner takes the fewest that fit the budget; a given layout must
        // fit as it is
        int32_t df;
        if (s.strassen_layout == 0) {
            df = strassen_choose_df(m, n, k, s.star_depth, s.strassen_depth, prec, s.tile, s.split_k,
                                    workspace_bytes);
            if (df < 0) return MM_ERR_WORKSPACE;
        } else {
            const int32_t mask = s.strassen_layout & ~MM_STRASSEN_LAYOUT_GIVEN;
            if (!(s.strassen_layout & MM_STRASSEN_LAYOUT_GIVEN) || mask < 0 || (mask >> s.strassen_depth) != 0)
                return MM_ERR_INVALID_ARG;
            if ((mask & (mask + 1)) != 0) return MM_ERR_UNSUPPORTED;  // depth-first levels must be the top ones
            df = 0;
            while ((mask >> df) & 1) ++df;
        }
        s.strassen_layout = MM_STRASSEN_LAYOUT((1 << df) - 1);
        const int64_t ws =
            star_strassen_ws_bytes(m, n, k, s.star_depth, s.strassen_depth, prec, s.tile, s.split_k, df);
        if (ws > (int64_t)workspace_bytes) return MM_ERR_WORKSPACE;
        mm_plan_info& pi = plan->info;
        pi.sched = s;
        pi.tile_k = tile_k_for(fam);
        pi.sar_levels = ilog2(s.split_k);
        pi.tar_levels = s.star_depth;
        pi.bands = m == 0 ? 0 : 1;
        pi.leaf_m = leaf_dim(m, s.strassen_depth + s.star_depth);
        pi.leaf_n = leaf_dim(n, s.strassen_depth + s.star_depth);
        pi.leaf_k = leaf_dim(k, s.strassen_depth + s.star_depth);
        pi.leaves = 1;
        for (int d = 0; d < s.strassen_depth; ++d) pi.leaves *= 7;
        for (int d = 0; d < s.star_depth; ++d) pi.leaves *= 8;
        const int t = s.tile ? s.tile : 128;
        pi.tiles_m = ceil_div(pi.leaf_m, t);
        pi.tiles_n = ceil_div(pi.leaf_n, t);
        // workgroups of one leaf launch: the leaves of one depth-first round
        int64_t round_leaves = 1;
        for (int d = df; d < s.strassen_depth; ++d) round_leaves *= 7;
        pi.workgroups = pi.tiles_m * pi.tiles_n * s.split_k * round_leaves;
        pi.ws_bytes = ws;
        plan->family = fam;
        plan->band_rows = std::max<int64_t>(m, 1);
        return MM_OK;
    }
    if (s.strassen_layout != 0 && s.strassen_layout != MM_STRASSEN_LAYOUT_GIVEN) return MM_ERR_INVALID_ARG;
    if (!exact && s.star_depth > 0 && !(s.flags & MM_FLAG_NONDETERMINISTIC))
        return MM_ERR_INVALID_ARG;

    if (s.flags & MM_FLAG_PERSISTENT) {
        // One persistent launch (SAR with per-tile arrival counters, Sec.
        // sar-mm): the slot ring holds a fixed number of tiles' partials,
        // whatever the problem size.
        if (s.star_depth != 0 || s.band_rows != 0) return MM_ERR_INVALID_ARG;
        if (s.tile == 0) s.tile = (int32_t)default_tile(m, n);
        if (!valid_tile(s.tile)) return MM_ERR_INVALID_ARG;
        const int tk = tile_k_for(fam);
        const int64_t tiles = ceil_div(m, s.tile) * ceil_div(n, s.tile);
        if (s.split_k == 0) {
            int64_t sk = 1;
            while (sk < kMaxSplit && tiles * sk < 2 * kCUs && ceil_div(k, tk) >= 16 * sk) sk *= 2;
            s.split_k = (int32_t)sk;
        }
        if (!is_pow2(s.split_k) || s.split_k > kMaxSplit) return MM_ERR_INVALID_ARG;
        // min{P, blocks} (Sec. sar-mm): never more slot groups than output tiles
        const int64_t groups = std::min<int64_t>(persist_groups(s.split_k), tiles);
        const int64_t ws =
            empty ? 0 : persist_ctl_bytes(groups) + groups * s.split_k * (int64_t)s.tile * s.tile * 4;
        if (ws > (int64_t)workspace_bytes) return MM_ERR_WORKSPACE;
        mm_plan_info& pi = plan->info;
        pi.sched = s;
        pi.tile_k = tk;
        pi.sar_levels = ilog2(s.split_k);
        pi.bands = m == 0 ? 0 : 1;
        pi.tiles_m = ceil_div(m, s.tile);
        pi.tiles_n = ceil_div(n, s.tile);
        pi.workgroups = tiles * s.split_k;  // (tile, slice) items
        pi.temp_elems = groups * s.split_k * (int64_t)s.tile * s.tile;
        pi.ws_bytes = ws;
        pi.leaf_m = m;
        pi.leaf_n = n;
        pi.leaf_k = k;
        pi.leaves = 1;
        plan->family = fam;
        plan->band_rows = std::max<int64_t>(m, 1);
        plan->persistent = true;
        plan->groups = groups;
        return MM_OK;
    }

    // Tile (the base case of the recursion).
    if (s.tile == 0) s.tile = (int32_t)default_tile(m, n);
    if (!valid_tile_for(fam, s.tile)) return MM_ERR_INVALID_ARG;
    const int tk = tile_k_for(fam);
    const int64_t kblocks = ceil_div(k, tk);
    const int64_t tiles_m_all = ceil_div(m, s.tile), tiles_n = ceil_div(n, s.tile);
    const size_t esz = c_elem_size(dt);
    const int64_t ldt = round_up(std::max<int64_t>(n, 1), 4);

    // k-split.
    const bool planner_split = s.split_k == 0;
    if (planner_split) {
        int64_t sk = 1;
        const int64_t tiles = tiles_m_all * tiles_n;
        if (s.tile >= 256) {
            // one 256 tile per CU (its stages take most of the LDS), so the
            // launch runs in whole rounds of kCUs workgroups: take the split
            // with the fewest rounds per unit of k (a larger split only when
            // it saves a tenth), 16 k-blocks per slice at least
            double best = (double)ceil_div(tiles, kCUs);
            for (int64_t c = 2; c <= kMaxSplit && kblocks >= 16 * c; c *= 2) {
                const double cost = (double)ceil_div(tiles * c, kCUs) / (double)c;
                if (cost < 0.9 * best) {
                    best = cost;
                    sk = c;
                }
            }
        } else {
            while (sk < kMaxSplit && tiles * sk < 2 * kCUs && kblocks >= 16 * sk) sk *= 2;
        }
        s.split_k = (int32_t)sk;
        s.star_depth = 0;
    }
    if (!is_pow2(s.split_k) || s.split_k > kMaxSplit) return MM_ERR_INVALID_ARG;
    int levels = ilog2(s.split_k);
    if (s.star_depth > levels) return MM_ERR_INVALID_ARG;

    // Temporaries: one per (TAR group, non-zero SAR index), each band_rows x ldt.
    auto temps_per_row = [&](int star) -> int64_t {
        if (empty) return 0;
        const int64_t groups = int64_t(1) << star;
        const int64_t per_group = (int64_t(1) << (levels - star)) - 1;
        return groups * per_group * ldt;  // elements per band row
    };
    int64_t band = s.band_rows;
    if (band != 0 && band < m && band % s.tile != 0) return MM_ERR_INVALID_ARG;

    auto fit_band = [&](int star) -> int64_t {
        // Largest band (whole tiles, at most m) whose temporaries fit the budget.
        const int64_t per_row = temps_per_row(star);
        if (per_row == 0 || m == 0) return std::max<int64_t>(m, 1);
        const int64_t rows = (int64_t)(workspace_bytes / esz) / per_row;
        if (rows >= m) return m;
        return (rows / s.tile) * s.tile;  // 0 if not even one tile row fits
    };

    if (band == 0) {
        band = fit_band(s.star_depth);
        if (band == 0 && planner_split) {
            // The budget cannot hold one band of temporaries.  Exact
            // semirings fall back to TAR merging (no temporaries); floats
            // reduce the split until it fits (s = 1 needs none).
            if (exact) {
                s.star_depth = levels;
                band = fit_band(s.star_depth);
            } else {
                while (band == 0 && s.split_k > 1) {
                    s.split_k /= 2;
                    levels = ilog2(s.split_k);
                    band = fit_band(0);
                }
            }
        }
        if (band == 0) return MM_ERR_WORKSPACE;
    }
    band = std::min<int64_t>(band, std::max<int64_t>(m, 1));
    const int levels_final = ilog2(s.split_k);
    const int64_t temp_elems = temps_per_row(s.star_depth) * band;
    if ((int64_t)(temp_elems * esz) > (int64_t)workspace_bytes) return MM_ERR_WORKSPACE;
    s.band_rows = band;

    // BF16x3: split the operands once into bf16 hi/lo planes (B transposed)
    // when the budget holds them beside the temporaries; the tile kernel then
    // stages plain copies.  Otherwise split inside the tile kernel.
    plan->planes = false;
    plan->ldp = plane_ld(k);
    plan->planes_bytes = 0;
    plan->temps_off = 0;
    int64_t ws_total = temp_elems * (int64_t)esz;
    // bf16 / fp16 inputs: copied once into one plane each for the 256- and
    // 128-wide direct-to-LDS tiles, when the budget holds them.
    const bool one_plane = (fam == KF_BF16_MFMA || fam == KF_F16_MFMA) && (s.tile == 256 || s.tile == 128);
    if ((fam == KF_BF16X3_MFMA || one_plane) && !(s.flags & MM_FLAG_SPLIT_IN_KERNEL) && !empty) {
        const int64_t pb =
            (int64_t)round_up((plane_rows(m) + plane_rows(n)) * plan->ldp * (one_plane ? 2 : 4), kAlign);
        if (pb + ws_total <= (int64_t)workspace_bytes) {
            plan->planes = true;
            plan->planes_bytes = pb;
            plan->temps_off = pb;
            ws_total += pb;
        }
    }

    mm_plan_info& pi = plan->info;
    pi.sched = s;
    pi.tile_k = tk;
    pi.tar_levels = s.star_depth;
    pi.sar_levels = levels_final - s.star_depth;
    pi.bands = m == 0 ? 0 : ceil_div(m, band);
    pi.tiles_m = ceil_div(band, s.tile);
    pi.tiles_n = tiles_n;
    pi.workgroups = pi.tiles_m * tiles_n * s.split_k;
    pi.temp_elems = temp_elems;
    pi.ws_bytes = ws_total;
    pi.leaf_m = m;
    pi.leaf_n = n;
    pi.leaf_k = k;
    pi.leaves = 1;
    plan->family = fam;
    plan->band_rows = band;
    plan->ldt = ldt;
    plan->temp_stride = band * ldt;
    return MM_OK;
}

}  // namespace starmm
