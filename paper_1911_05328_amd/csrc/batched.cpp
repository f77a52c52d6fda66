// Host side of the batched launch: validation, per-problem schedule, the
// cost-sorted work list, the workspace layout (tables, counters, split-K
// slots, packed operand planes), and the optional hipGraph that captures the
// persistent kernel (for fp32 operands, the pack kernel before it).
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "batched.hpp"
#include "internal.hpp"

namespace starmm {

namespace {

struct BatchLayout {
    std::vector<BatchProblem> probs;
    std::vector<BatchItem> items;                // the tiles of each kernel kind, kind by kind
    int64_t kind_begin[kBatchKinds + 1] = {};    // items of kind j: [kind_begin[j], kind_begin[j + 1])
    BatchQueues queues[kBatchKinds] = {};        // per-XCD queues inside each kind's list
    std::vector<BatchItem> pack;                 // pack work list: (problem, block), problems in work order
    std::vector<int64_t> ap_off, bp_off;         // plane offsets (bytes) inside the planes region
    int64_t off_ctl = 0, off_probs = 0, off_items = 0, off_counters = 0, off_temps = 0, off_pack = 0,
            off_packdone = 0, off_planes = 0, bytes = 0;
    int64_t n_counters = 0, n_temps = 0, plane_bytes = 0;
};

mm_status build_layout(int32_t count, const mm_problem* problems, mm_dtype dt, const mm_schedule* scheds,
                       BatchLayout* L) {
    if (count < 0 || (count > 0 && !problems)) return MM_ERR_INVALID_ARG;
    if (dt != MM_DT_BF16 && dt != MM_DT_F16 && dt != MM_DT_F32) return MM_ERR_UNSUPPORTED;
    if ((int64_t)count > (int64_t)UINT32_MAX) return MM_ERR_INVALID_ARG;
    const int T = batched_tile(), TW = batched_wide_tile();
    const size_t esz = dt == MM_DT_F32 ? 4 : 2;
    const int64_t align_elems = dt == MM_DT_F32 ? 4 : 8;
    L->probs.resize(count);
    std::vector<int64_t> cost(count);
    for (int32_t i = 0; i < count; ++i) {
        const mm_problem& q = problems[i];
        if (q.m < 0 || q.n < 0 || q.k < 0) return MM_ERR_INVALID_ARG;
        if (q.lda < std::max<int64_t>(q.k, 1) || q.ldb < std::max<int64_t>(q.n, 1) ||
            q.ldc < std::max<int64_t>(q.n, 1))
            return MM_ERR_INVALID_ARG;
        if ((q.m > 0 && q.k > 0 && !q.A) || (q.k > 0 && q.n > 0 && !q.B) || (q.m > 0 && q.n > 0 && !q.C))
            return MM_ERR_INVALID_ARG;
        int32_t split = 1, tile = 0;
        bool pack = true, overwrite = false;
        if (scheds) {
            const mm_schedule& s = scheds[i];
            if (s.strassen_depth != 0) return MM_ERR_UNSUPPORTED;
            if (s.tile != 0 && s.tile != T && s.tile != TW) return MM_ERR_UNSUPPORTED;
            if (s.star_depth != 0 || s.band_rows != 0 ||
                (s.flags & ~(MM_FLAG_SPLIT_IN_KERNEL | MM_FLAG_OVERWRITE_C)) != 0)
                return MM_ERR_INVALID_ARG;
            split = s.split_k == 0 ? 1 : s.split_k;
            if (!is_pow2(split) || split > kMaxSplit) return MM_ERR_INVALID_ARG;
            pack = !(s.flags & MM_FLAG_SPLIT_IN_KERNEL);
            overwrite = (s.flags & MM_FLAG_OVERWRITE_C) != 0;
            tile = s.tile;
            if (tile == TW && !pack) return MM_ERR_UNSUPPORTED;  // wide tiles read packed planes only
        }
        if (tile == 0) {
            // Wide tiles (twice the operand reuse per copied byte) for every
            // packed problem, narrow ones included: in the 512-problem batch
            // that measured 2% faster (3.07 against 3.14 ms) than keeping
            // problems narrower than 256 on 128 tiles, which in turn was 2%
            // faster than also requiring k >= 1024; it also leaves one
            // persistent kernel for the whole packed batch.
            tile = pack ? TW : T;
        }
        // a problem with nothing to pack (k = 0) runs on the staged 128 tiles
        if (!(pack && q.m > 0 && q.n > 0 && q.k > 0)) tile = T;
        BatchProblem& p = L->probs[i];
        p.m = q.m;
        p.n = q.n;
        p.k = q.k;
        p.A = q.A;
        p.lda = q.lda;
        p.B = q.B;
        p.ldb = q.ldb;
        p.C = q.C;
        p.ldc = q.ldc;
        p.tile = tile;
        p.tiles_m = ceil_div(q.m, tile);
        p.tiles_n = ceil_div(q.n, tile);
        p.levels = ilog2(split);
        // 16-byte aligned rows take plain vector loads, others the funnel-shift path
        p.vec_ok = (q.lda % align_elems == 0) && (q.ldb % align_elems == 0) && ((uintptr_t)q.A % 16 == 0) &&
                   ((uintptr_t)q.B % 16 == 0);
        p.temp_off = 0;
        p.counter_off = 0;
        p.packed = pack && q.m > 0 && q.n > 0 && q.k > 0;
        p.overwrite = overwrite ? 1 : 0;
        p.kind = !p.packed ? 0 : (tile == TW ? 2 : 1);
        p.ap = p.bp = nullptr;
        p.lp = p.a_plane = p.b_plane = 0;
        cost[i] = (q.m == 0 || q.n == 0) ? 0 : p.tiles_m * p.tiles_n * std::max<int64_t>(ceil_div(q.k, kBf16BKHost), 1);
        (void)esz;
    }
    // Packed operands: k-tiled planes (one for bf16 / fp16 inputs, hi/lo for fp32)
    // in the workspace, and the pack kernel's work list.
    const int64_t np = dt == MM_DT_F32 ? 2 : 1;
    L->ap_off.assign(count, 0);
    L->bp_off.assign(count, 0);
    for (int32_t i = 0; i < count; ++i) {
        BatchProblem& p = L->probs[i];
        if (p.packed) {
            p.lp = plane_ld(p.k);
            p.a_plane = plane_rows(p.m) * p.lp;
            p.b_plane = plane_rows(p.n) * p.lp;
            L->ap_off[i] = L->plane_bytes;
            L->plane_bytes = round_up(L->plane_bytes + np * p.a_plane * 2, kAlign);
            L->bp_off[i] = L->plane_bytes;
            L->plane_bytes = round_up(L->plane_bytes + np * p.b_plane * 2, kAlign);
            const int64_t kb = ceil_div(p.lp, batched_pack_k()), R = batched_pack_rows();
            const int64_t blocks = (ceil_div(plane_rows(p.m), R) + ceil_div(plane_rows(p.n), R)) * kb;
            if (blocks > INT32_MAX) return MM_ERR_INVALID_ARG;
            p.pack_blocks = (int32_t)blocks;
        } else {
            p.pack_blocks = 0;
        }
        p.reserved = 0;
    }
    // Longest work first: items of costlier problems come earlier in the list.
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const BatchProblem &pa = L->probs[a], &pb = L->probs[b];
        const int64_t ka = ceil_div(pa.k, int64_t(1) << pa.levels), kb2 = ceil_div(pb.k, int64_t(1) << pb.levels);
        return ka != kb2 ? ka > kb2 : cost[a] > cost[b];
    });
    // Each problem's items (tile-major in the recursion's tile order, slices
    // of a tile adjacent) are cut into chunks of the tiles one XCD runs at
    // once; chunks go to the least-loaded XCD queue of their kind, longest
    // first, so neighbouring tiles share that XCD's L2.
    std::vector<BatchItem> lists[kBatchKinds][kBatchQueues];
    int64_t load[kBatchKinds][kBatchQueues] = {};
    const int64_t chunk_tiles[kBatchKinds] = {64, 64, 32};  // resident tiles per XCD of each kind
    int64_t n_items = 0;
    // the pack list follows the same order, so the first tiles' planes are
    // the first packed
    for (int32_t idx : order) {
        const BatchProblem& p = L->probs[idx];
        if ((int64_t)L->pack.size() + p.pack_blocks > (int64_t)UINT32_MAX) return MM_ERR_INVALID_ARG;
        for (int64_t b = 0; b < p.pack_blocks; ++b) L->pack.push_back(BatchItem{(uint32_t)idx, (uint32_t)b});
    }
    for (int32_t idx : order) {
        BatchProblem& p = L->probs[idx];
        // (k = 0 still writes C = 0 when C is overwritten)
        if (p.m == 0 || p.n == 0 || (p.k == 0 && !p.overwrite)) continue;
        const int64_t tiles = p.tiles_m * p.tiles_n, s = int64_t(1) << p.levels;
        if (s > 1) {
            p.counter_off = L->n_counters;
            p.temp_off = L->n_temps;
            L->n_counters += tiles;
            L->n_temps += tiles * s * p.tile * p.tile;
        }
        if (n_items + tiles * s > (int64_t)UINT32_MAX) return MM_ERR_INVALID_ARG;
        n_items += tiles * s;
        const int64_t ct = chunk_tiles[p.kind], ksteps = std::max<int64_t>(ceil_div(p.k, kBf16BKHost), 1);
        for (int64_t t0 = 0; t0 < tiles; t0 += ct) {
            const int64_t t1 = std::min(tiles, t0 + ct);
            int q = 0;
            for (int j = 1; j < kBatchQueues; ++j)
                if (load[p.kind][j] < load[p.kind][q]) q = j;
            load[p.kind][q] += (t1 - t0) * ksteps;
            for (int64_t u = t0 * s; u < t1 * s; ++u) lists[p.kind][q].push_back(BatchItem{(uint32_t)idx, (uint32_t)u});
        }
    }
    for (int j = 0; j < kBatchKinds; ++j) {
        L->kind_begin[j] = (int64_t)L->items.size();
        for (int q = 0; q < kBatchQueues; ++q) {
            L->queues[j].begin[q] = (uint32_t)((int64_t)L->items.size() - L->kind_begin[j]);
            L->items.insert(L->items.end(), lists[j][q].begin(), lists[j][q].end());
        }
        L->queues[j].begin[kBatchQueues] = (uint32_t)((int64_t)L->items.size() - L->kind_begin[j]);
    }
    L->kind_begin[kBatchKinds] = (int64_t)L->items.size();
    L->off_ctl = 0;  // one counter block per queue of each kernel kind
    L->off_probs = round_up(kBatchKinds * kBatchQueues * sizeof(BatchCtl), kAlign);
    L->off_items = round_up(L->off_probs + (int64_t)(count * sizeof(BatchProblem)), kAlign);
    L->off_counters = round_up(L->off_items + (int64_t)(L->items.size() * sizeof(BatchItem)), kAlign);
    L->off_temps = round_up(L->off_counters + L->n_counters * 4, kAlign);
    L->off_pack = round_up(L->off_temps + L->n_temps * 4, kAlign);
    L->off_packdone = round_up(L->off_pack + (int64_t)(L->pack.size() * sizeof(BatchItem)), kAlign);
    L->off_planes = round_up(L->off_packdone + (int64_t)count * 4, kAlign);
    L->bytes = round_up(L->off_planes + L->plane_bytes, kAlign);
    return MM_OK;
}

// Upload the tables (with the plane pointers of this workspace) and clear
// the counters, in stream order.
mm_status upload(const BatchLayout& L, void* ws, hipStream_t st) {
    char* w = static_cast<char*>(ws);
    std::vector<BatchProblem> probs = L.probs;
    for (size_t i = 0; i < probs.size(); ++i)
        if (probs[i].packed) {
            probs[i].ap = reinterpret_cast<const uint16_t*>(w + L.off_planes + L.ap_off[i]);
            probs[i].bp = reinterpret_cast<const uint16_t*>(w + L.off_planes + L.bp_off[i]);
        }
    hipError_t e = hipMemsetAsync(w + L.off_ctl, 0, kBatchKinds * kBatchQueues * sizeof(BatchCtl), st);
    if (e == hipSuccess && !probs.empty())
        e = hipMemcpyAsync(w + L.off_probs, probs.data(), probs.size() * sizeof(BatchProblem),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !L.pack.empty())
        e = hipMemcpyAsync(w + L.off_pack, L.pack.data(), L.pack.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                           st);
    if (e == hipSuccess && !L.items.empty())
        e = hipMemcpyAsync(w + L.off_items, L.items.data(), L.items.size() * sizeof(BatchItem),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess && L.n_counters > 0) e = hipMemsetAsync(w + L.off_counters, 0, L.n_counters * 4, st);
    if (e == hipSuccess && !probs.empty()) e = hipMemsetAsync(w + L.off_packdone, 0, probs.size() * 4, st);
    if (e != hipSuccess) {
        set_last_error(std::string("batched upload: ") + hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    return MM_OK;
}

// Tile mode of a batch dtype: 0 fp32 (BF16x3 split), 1 bf16, 5 fp16.
int batched_mode(mm_dtype dt) { return dt == MM_DT_F32 ? 0 : (dt == MM_DT_F16 ? 5 : 1); }

hipError_t launch_from(const BatchLayout& L, int mode, void* ws, hipStream_t st) {
    char* w = static_cast<char*>(ws);
    const auto* probs = reinterpret_cast<const BatchProblem*>(w + L.off_probs);
    const auto* items = reinterpret_cast<const BatchItem*>(w + L.off_items);
    auto* ctl = reinterpret_cast<BatchCtl*>(w + L.off_ctl);
    auto* counters = reinterpret_cast<uint32_t*>(w + L.off_counters);
    auto* temps = reinterpret_cast<float*>(w + L.off_temps);
    const auto* pack_list = reinterpret_cast<const BatchItem*>(w + L.off_pack);
    auto* pack_done = reinterpret_cast<uint32_t*>(w + L.off_packdone);
    const uint32_t npack = (uint32_t)L.pack.size(), nprob = (uint32_t)L.probs.size();
    hipError_t e = hipSuccess;
    // fp32 operands are split by a pack kernel of their own; bf16 / fp16
    // ones are packed by the wide kind's launch (launched for that alone if
    // it has no tiles), which runs first
    const bool fused = batched_fused_pack(mode);
    if (!fused) e = launch_batched_pack(mode, probs, pack_list, (int64_t)npack, st);
    // the wide tiles (the most work) first, then the narrow packed ones,
    // then problems staged from their operands
    for (int kind : {2, 1, 0}) {
        const int64_t b = L.kind_begin[kind], cnt = L.kind_begin[kind + 1] - b;
        const bool packs = fused && kind == 2 && npack > 0;
        if (e != hipSuccess || (cnt == 0 && !packs)) continue;
        const int64_t work = std::max<int64_t>(cnt, packs ? (int64_t)npack : 0);
        e = launch_batched(mode, kind, (int)std::min<int64_t>(batched_grid(mode, kind), work), probs, items + b,
                           L.queues[kind], ctl + kind * kBatchQueues, counters, temps, st,
                           packs ? pack_list : nullptr, packs ? npack : 0u, packs ? pack_done : nullptr, nprob);
    }
    return e;
}

}  // namespace

}  // namespace starmm

using namespace starmm;

struct mm_batched_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

size_t mm_batched_workspace_bytes(int32_t count, const mm_problem* problems, mm_dtype dt, const mm_schedule* scheds) {
    BatchLayout L;
    if (build_layout(count, problems, dt, scheds, &L) != MM_OK) return 0;
    return (size_t)L.bytes;
}

mm_status mm_batched(int32_t count, const mm_problem* problems, mm_dtype dt, const mm_schedule* scheds,
                     void* workspace, size_t workspace_bytes, void* stream) {
    BatchLayout L;
    mm_status st = build_layout(count, problems, dt, scheds, &L);
    if (st != MM_OK) return st;
    if (L.items.empty()) return MM_OK;
    if (!workspace_ok(workspace, workspace_bytes)) return MM_ERR_INVALID_ARG;
    if (!workspace || (int64_t)workspace_bytes < L.bytes) return MM_ERR_WORKSPACE;
    const int mode = batched_mode(dt);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload(L, workspace, s)) != MM_OK) return st;
    hipError_t e = launch_from(L, mode, workspace, s);
    if (e != hipSuccess) {
        set_last_error(std::string("mm_batched launch: ") + hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    return MM_OK;
}

mm_status mm_batched_graph_create(int32_t count, const mm_problem* problems, mm_dtype dt, const mm_schedule* scheds,
                                  void* workspace, size_t workspace_bytes, void* stream, mm_batched_graph** out) {
    if (!out) return MM_ERR_INVALID_ARG;
    *out = nullptr;
    BatchLayout L;
    mm_status st = build_layout(count, problems, dt, scheds, &L);
    if (st != MM_OK) return st;
    if (!workspace_ok(workspace, workspace_bytes)) return MM_ERR_INVALID_ARG;
    if (!workspace || (int64_t)workspace_bytes < L.bytes) return MM_ERR_WORKSPACE;
    const int mode = batched_mode(dt);
    hipStream_t s = (hipStream_t)stream;
    if ((st = upload(L, workspace, s)) != MM_OK) return st;
    hipError_t e = hipStreamSynchronize(s);
    hipStream_t cap = nullptr;
    auto* g = new mm_batched_graph();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_from(L, mode, workspace, cap);
        e = hipStreamEndCapture(cap, &g->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        set_last_error(std::string("mm_batched_graph_create: ") + hipGetErrorString(e));
        if (g->exec) hipGraphExecDestroy(g->exec);
        if (g->graph) hipGraphDestroy(g->graph);
        delete g;
        return MM_ERR_HIP;
    }
    *out = g;
    return MM_OK;
}

mm_status mm_batched_graph_launch(mm_batched_graph* g, void* stream) {
    if (!g || !g->exec) return MM_ERR_INVALID_ARG;
    ProfScope ps("batched_graph", (hipStream_t)stream);
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_last_error(std::string("mm_batched_graph_launch: ") + hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    return MM_OK;
}

void mm_batched_graph_destroy(mm_batched_graph* g) {
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
