// Schedule selection for calls that pass no schedule, once the caller has
// loaded a cost model and/or measured timings: a measured best for the exact
// problem first, else the cost model's proposal, else the built-in planner.
//
// The cost model is the MLP trained on the autotuner's timings (inputs:
// log2 m, n, k / 14, dtype one-hot, log2(budget / |C|) / 3; three hidden
// layers of 64 ReLU units; one standardised natural-log time per schedule).
// Its schedule space is Strassen depth 0-3 x k-split 1, 2, 4, 8 x tile 32,
// 64, 128, 256 (fp32 products through the BF16x3 split with Winograd levels,
// products without Strassen as one band of C).  Its proposal is the argmin of
// the predicted times over the schedules the planner accepts for the budget.
// Pure host code, evaluated in double.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace starmm {

namespace {

constexpr int kIn = 7, kHid = 64, kOut = 64;
constexpr int kDepths[4] = {0, 1, 2, 3}, kSplits[4] = {1, 2, 4, 8}, kTiles[4] = {32, 64, 128, 256};
constexpr size_t kMemoMax = 4096;

struct CostModel {
    double t_mean = 0.0, t_std = 1.0;
    std::vector<double> W[4], b[4];  // W[l] is out x in, row-major
    bool accurate[3][kOut] = {};     // per space dtype: schedule measured within the error target
};

using ShapeKey = std::tuple<int, int, int64_t, int64_t, int64_t>;          // sr, dt, m, n, k
using CallKey = std::tuple<int, int, int64_t, int64_t, int64_t, uint64_t>;  // + budget

struct Selector {
    bool has_model = false;
    CostModel model;
    std::map<ShapeKey, std::vector<mm_tuned_entry>> db;
    std::map<CallKey, std::pair<bool, mm_schedule>> memo;  // (chosen?, schedule)
};

std::mutex g_mu;
Selector g_sel;

int64_t weight_count() { return 2 + kHid * kIn + kHid + 2 * (kHid * kHid + kHid) + kOut * kHid + kOut; }
// the weights, then the accuracy mask (3 dtypes x kOut schedules, 1 = acceptable)
int64_t param_count() { return weight_count() + 3 * kOut; }

// The space's dtype index of a (semiring, dtype) pair: 0 fp32 through the
// split path, 1 bf16 inputs, 2 int32 (min,+); -1 outside the space.
int space_dtype(mm_semiring_kind sr, mm_dtype dt) {
    if (sr == MM_SR_PLUS_TIMES && dt == MM_DT_F32) return 0;
    if (sr == MM_SR_PLUS_TIMES && dt == MM_DT_BF16) return 1;
    if (sr == MM_SR_MIN_PLUS && dt == MM_DT_I32) return 2;
    return -1;
}

mm_schedule space_schedule(int idx, int sdt, int64_t m) {
    const int d = kDepths[idx / 16], s = kSplits[(idx / 4) % 4], t = kTiles[idx % 4];
    mm_schedule sc;
    std::memset(&sc, 0, sizeof sc);
    sc.tile = t;
    sc.split_k = s;
    sc.strassen_depth = d;
    sc.variant = MM_STRASSEN_WINOGRAD;
    // fp32 to fp32 accuracy: BF16x3 without Strassen levels, FP16x3 under them
    sc.precision = sdt != 0 ? MM_PREC_F32 : (d == 0 ? MM_PREC_BF16X3 : MM_PREC_FP16X3);
    sc.band_rows = d > 0 ? 0 : std::max<int64_t>(m, 1);
    // Strassen levels breadth-first, as they were timed
    sc.strassen_layout = d > 0 ? MM_STRASSEN_LAYOUT(0) : 0;
    return sc;
}

// Predicted natural-log milliseconds of every schedule of the space.
void predict(const CostModel& cm, int sdt, int64_t m, int64_t n, int64_t k, size_t budget, double* out) {
    const double rel = std::max((double)budget, 1.0) / ((double)m * (double)n * 4.0);
    std::vector<double> cur = {std::log2((double)m) / 14.0, std::log2((double)n) / 14.0,
                               std::log2((double)k) / 14.0, sdt == 0 ? 1.0 : 0.0, sdt == 1 ? 1.0 : 0.0,
                               sdt == 2 ? 1.0 : 0.0, std::log2(rel) / 3.0};
    std::vector<double> nxt;
    for (int l = 0; l < 4; ++l) {
        const int in = (int)cur.size(), o = (int)cm.b[l].size();
        nxt.assign(o, 0.0);
        for (int r = 0; r < o; ++r) {
            double acc = cm.b[l][r];
            for (int c = 0; c < in; ++c) acc += cm.W[l][(size_t)r * in + c] * cur[c];
            nxt[r] = (l < 3 && acc < 0.0) ? 0.0 : acc;
        }
        cur.swap(nxt);
    }
    for (int j = 0; j < kOut; ++j) out[j] = cur[j] * cm.t_std + cm.t_mean;
}

bool fits(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, size_t budget,
          const mm_schedule& sc, Plan* p) {
    return make_plan(sr, dt, m, n, k, budget, &sc, p) == MM_OK;
}

// The model's proposal (false when the pair is outside the space or nothing fits).
bool model_pick(const CostModel& cm, mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                size_t budget, mm_schedule* out, double* pred_ms) {
    const int sdt = space_dtype(sr, dt);
    if (sdt < 0 || m <= 0 || n <= 0 || k <= 0) return false;
    double pred[kOut];
    predict(cm, sdt, m, n, k, budget, pred);
    int best = -1;
    for (int j = 0; j < kOut; ++j) {
        if (!cm.accurate[sdt][j]) continue;  // measured above the error target
        Plan p;
        if (!fits(sr, dt, m, n, k, budget, space_schedule(j, sdt, m), &p)) continue;
        if (best < 0 || pred[j] < pred[best]) best = j;
    }
    if (best < 0) return false;
    *out = space_schedule(best, sdt, m);
    if (pred_ms) *pred_ms = std::exp(pred[best]);
    return true;
}

// The fastest measured schedule for the exact problem that runs, within the
// budget, as it was timed: a schedule timed over operand planes (BF16x3
// without Strassen levels; bf16 inputs on 128- and 256-wide tiles) counts
// only where the planes fit (the planner would otherwise split or stage
// inside the kernel, a different timing).
bool db_pick(const Selector& sel, mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
             size_t budget, mm_schedule* out, double* ms) {
    auto it = sel.db.find(ShapeKey((int)sr, (int)dt, m, n, k));
    if (it == sel.db.end()) return false;
    const mm_tuned_entry* best = nullptr;
    for (const mm_tuned_entry& e : it->second) {
        Plan p;
        if (!fits(sr, dt, m, n, k, budget, e.sched, &p)) continue;
        // timed over operand planes, but the budget would not hold them
        const bool plane_timed =
            !(e.sched.flags & MM_FLAG_SPLIT_IN_KERNEL) &&
            ((p.family == KF_BF16X3_MFMA && e.sched.strassen_depth == 0 && !prec_fp16(e.sched.precision)) ||
             ((p.family == KF_BF16_MFMA || p.family == KF_F16_MFMA) &&
              (e.sched.tile == 128 || e.sched.tile == 256)));
        if (plane_timed && !p.planes) continue;
        if (!best || e.ms < best->ms) best = &e;
    }
    if (!best) return false;
    *out = best->sched;
    if (ms) *ms = best->ms;
    return true;
}

}  // namespace

bool select_schedule(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k, size_t budget,
                     mm_schedule* out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_sel.has_model && g_sel.db.empty()) return false;
    const CallKey key((int)sr, (int)dt, m, n, k, (uint64_t)budget);
    auto it = g_sel.memo.find(key);
    if (it != g_sel.memo.end()) {
        if (it->second.first) *out = it->second.second;
        return it->second.first;
    }
    mm_schedule sc;
    std::memset(&sc, 0, sizeof sc);
    bool ok = db_pick(g_sel, sr, dt, m, n, k, budget, &sc, nullptr);
    if (!ok && g_sel.has_model) ok = model_pick(g_sel.model, sr, dt, m, n, k, budget, &sc, nullptr);
    if (g_sel.memo.size() >= kMemoMax) g_sel.memo.clear();
    g_sel.memo[key] = {ok, sc};
    if (ok) *out = sc;
    return ok;
}

}  // namespace starmm

using namespace starmm;

extern "C" {

int64_t mm_cost_model_param_count(void) { return param_count(); }

mm_status mm_cost_model_load(const float* params, int64_t count) {
    if (!params || count != param_count()) return MM_ERR_INVALID_ARG;
    CostModel cm;
    const float* q = params;
    cm.t_mean = *q++;
    cm.t_std = *q++;
    if (!(cm.t_std > 0.0) || !std::isfinite(cm.t_std) || !std::isfinite(cm.t_mean)) return MM_ERR_INVALID_ARG;
    const int sizes[5] = {kIn, kHid, kHid, kHid, kOut};
    for (int l = 0; l < 4; ++l) {
        const int in = sizes[l], o = sizes[l + 1];
        cm.W[l].assign(q, q + (size_t)o * in);
        q += (size_t)o * in;
        cm.b[l].assign(q, q + o);
        q += o;
    }
    for (int l = 0; l < 4; ++l)
        for (double v : cm.W[l])
            if (!std::isfinite(v)) return MM_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < kOut; ++j) {
            const float v = *q++;
            if (v != 0.0f && v != 1.0f) return MM_ERR_INVALID_ARG;
            cm.accurate[d][j] = v == 1.0f;
        }
    std::lock_guard<std::mutex> lock(g_mu);
    g_sel.model = std::move(cm);
    g_sel.has_model = true;
    g_sel.memo.clear();
    return MM_OK;
}

mm_status mm_tuned_load(const mm_tuned_entry* entries, int64_t count) {
    if (count < 0 || (count > 0 && !entries)) return MM_ERR_INVALID_ARG;
    std::map<ShapeKey, std::vector<mm_tuned_entry>> db;
    for (int64_t i = 0; i < count; ++i) {
        const mm_tuned_entry& e = entries[i];
        if (e.m <= 0 || e.n <= 0 || e.k <= 0 || !(e.ms >= 0.0) || !std::isfinite(e.ms)) return MM_ERR_INVALID_ARG;
        Plan p;  // the schedule must be valid for its problem with some budget
        if (make_plan((mm_semiring_kind)e.semiring, (mm_dtype)e.dtype, e.m, e.n, e.k, ~size_t(0) >> 1, &e.sched,
                      &p) != MM_OK)
            return MM_ERR_INVALID_ARG;
        db[ShapeKey(e.semiring, e.dtype, e.m, e.n, e.k)].push_back(e);
    }
    std::lock_guard<std::mutex> lock(g_mu);
    g_sel.db = std::move(db);
    g_sel.memo.clear();
    return MM_OK;
}

void mm_schedule_selection_clear(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_sel = Selector();
}

mm_status mm_propose_schedule(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                              size_t workspace_bytes, mm_schedule* out, double* predicted_ms) {
    if (!out || m <= 0 || n <= 0 || k <= 0) return MM_ERR_INVALID_ARG;
    if (space_dtype(sr, dt) < 0) return MM_ERR_UNSUPPORTED;
    CostModel cm;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_sel.has_model) return MM_ERR_UNSUPPORTED;
        cm = g_sel.model;
    }
    mm_schedule sc;
    if (!model_pick(cm, sr, dt, m, n, k, workspace_bytes, &sc, predicted_ms)) return MM_ERR_WORKSPACE;
    *out = sc;
    return MM_OK;
}

mm_status mm_tuned_lookup(mm_semiring_kind sr, mm_dtype dt, int64_t m, int64_t n, int64_t k,
                          size_t workspace_bytes, mm_schedule* out, double* measured_ms) {
    if (!out) return MM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_mu);
    mm_schedule sc;
    if (!db_pick(g_sel, sr, dt, m, n, k, workspace_bytes, &sc, measured_ms)) return MM_ERR_UNSUPPORTED;
    *out = sc;
    return MM_OK;
}

}  // extern "C"
