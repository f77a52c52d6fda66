"""Batch-aware autotuner for mm_batched (not in the paper): chooses each
problem's schedule (tile edge, k-split) by timing the whole batch, since a
problem's best schedule inside a batch that already fills the GPU differs from
its best schedule launched alone (there a k-split buys parallelism; here it
mostly adds merge work, except for the few deep problems that would otherwise
form the launch's tail).

Problems are grouped into classes by their depth in k (the length of one
tile's pipeline) and their tile count; every class starts from the library's
own rule (split 1; packed operands on 256-wide tiles) and a coordinate
descent over the classes
(tile, k-split, packed or staged straight from the operands), heaviest first,
keeps a class's alternative when the whole batch, captured as one graph and
replayed, gets faster by more than the timing noise.  Strassen levels are
not in the space: for bf16 inputs a Strassen leaf needs its operand sums
split into hi/lo parts to keep the product's accuracy (a sum of two bf16
values is not a bf16 value), so one level costs 3 x 7 / 8 of the
classical bf16 product's MFMA work, and `strassen_check` times that on the
batch's largest problems.

Usage from Python: ``scheds, report = tune(triples)`` (triples of device
tensors A, B, C as for ``batched_mm``); the schedules go to ``BatchedGraph``
or ``batched_mm``.
"""
from __future__ import annotations

import math
import time

TILE_NARROW, TILE_WIDE = 128, 256


def problem_class(m: int, n: int, k: int) -> tuple:
    """(tile of the library's rule, k bucket, tile-count bucket); the rule
    gives every packed problem the wide tile."""
    t = TILE_WIDE
    kb = 0 if k < 512 else (1 if k < 2048 else 2)
    tiles = math.ceil(m / t) * math.ceil(n / t)
    tb = 0 if tiles < 4 else (1 if tiles < 32 else 2)
    return (t, kb, tb)


def options(cls: tuple) -> list:
    """(tile, split, packed) alternatives of a class; the first is the
    rule's.  packed: the operands are rewritten as k-tiled planes by the
    batch's pack kernel (the direct-to-LDS tiles read those); unpacked
    problems stage 128 tiles straight from their operands."""
    t, kb, _ = cls
    opts = [(t, 1, True)]
    for packed in (True, False):
        for tile in ((TILE_NARROW, TILE_WIDE) if packed else (TILE_NARROW,)):
            for split in (1, 2, 4, 8):
                if (tile, split, packed) == (t, 1, True):
                    continue
                if split > 1 and kb == 0:
                    continue  # a shallow pipeline gains nothing from splitting
                opts.append((tile, split, packed))
    return opts


def _schedule(sm, opt):
    tile, split, packed = opt
    return sm.make_schedule(tile=tile, split_k=split, flags=0 if packed else sm.FLAG_SPLIT_IN_KERNEL)


def _schedules(sm, shapes, choice):
    return [_schedule(sm, choice[problem_class(*s)]) for s in shapes]


def time_batch(sm, torch, triples, scheds, launches: int = 10, reps: int = 3) -> float:
    """Median over `reps` of the mean time of `launches` graph replays (ms)."""
    ws = torch.empty(max(sm.batched_workspace_bytes(triples, scheds), 1), dtype=torch.uint8, device="cuda")
    g = sm.BatchedGraph(triples, schedules=scheds, workspace=ws)
    try:
        for _ in range(2):
            g.launch()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(launches):
                g.launch()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / launches)
    finally:
        g.close()
    ts.sort()
    return ts[len(ts) // 2]


def tune(triples, noise: float = 0.01, passes: int = 2, log=None):
    """Per-problem schedules for the batch `triples` and a report:
    {"classes": {class: [tile, split]}, "baseline_ms", "tuned_ms", "evaluations", "trace"}."""
    import torch

    import paper_1911_05328_amd as sm

    shapes = [(int(A.shape[0]), int(B.shape[1]), int(A.shape[1])) for A, B, _ in triples]
    flops = {}
    for m, n, k in shapes:
        c = problem_class(m, n, k)
        flops[c] = flops.get(c, 0.0) + 2.0 * m * n * k
    order = sorted(flops, key=lambda c: -flops[c])
    choice = {c: options(c)[0] for c in order}
    t0 = time.perf_counter()
    best = time_batch(sm, torch, triples, _schedules(sm, shapes, choice))
    base = best
    trace = [{"class": None, "option": None, "ms": best}]
    evals = 1
    for _ in range(passes):
        improved = False
        for c in order:
            for opt in options(c):
                if opt == choice[c]:
                    continue
                trial = dict(choice)
                trial[c] = opt
                ms = time_batch(sm, torch, triples, _schedules(sm, shapes, trial))
                evals += 1
                trace.append({"class": list(c), "option": list(opt), "ms": ms})
                if ms < best * (1.0 - noise):
                    best, choice, improved = ms, trial, True
                    if log:
                        log(f"batch tuner: class {c} -> tile {opt[0]} split {opt[1]} packed {opt[2]}: "
                            f"{ms:.3f} ms")
        if not improved:
            break
    # re-time the final choice against the rule in alternation (drift check)
    final, rule = [], []
    rule_choice = {c: options(c)[0] for c in order}
    for _ in range(3):
        rule.append(time_batch(sm, torch, triples, _schedules(sm, shapes, rule_choice)))
        final.append(time_batch(sm, torch, triples, _schedules(sm, shapes, choice)))
    rule.sort()
    final.sort()
    report = {"classes": {str(list(c)): list(choice[c]) for c in order},
              "class_gflop": {str(list(c)): flops[c] / 1e9 for c in order},
              "search_baseline_ms": base, "search_best_ms": best,
              "rule_ms": rule[1], "tuned_ms": final[1], "evaluations": evals,
              "tuning_s": time.perf_counter() - t0, "trace": trace}
    return _schedules(sm, shapes, choice), report


def strassen_check(triples, count: int = 8):
    """For the `count` largest problems: the bf16 product alone (mm_semiring,
    bf16 inputs copied into planes, 256-wide direct-to-LDS tiles, the fastest
    of k-splits 1, 2 and 4) against
    one Strassen level over the BF16x3
    split product of the same values (mm_strassen on fp32 copies), the form
    that keeps the bf16 product's accuracy.  Times in ms (median of 5)."""
    import torch

    import paper_1911_05328_amd as sm

    def med(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        return ts[2]

    big = sorted(triples, key=lambda t: -t[0].shape[0] * t[1].shape[1] * t[0].shape[1])[:count]
    rows = []
    for A, B, C in big:
        m, k = A.shape
        n = B.shape[1]
        Cw = torch.zeros(m, n, device="cuda")
        t_bf16, split_bf16 = None, None
        for split in (1, 2, 4):
            s_bf = sm.make_schedule(tile=256, split_k=split)
            ws_bf = torch.empty(max(sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_BF16, m, n, k, s_bf), 1),
                                dtype=torch.uint8, device="cuda")
            t = med(lambda: sm.semiring_mm(A, B, Cw, sm.PLUS_TIMES, workspace=ws_bf, schedule=s_bf))
            if t_bf16 is None or t < t_bf16:
                t_bf16, split_bf16 = t, split
            del ws_bf
        A32, B32 = A.float(), B.float()
        ws = torch.empty(sm.strassen_workspace_bytes(m, n, k, 1, sm.CLASSIC, sm.PREC_BF16X3), dtype=torch.uint8,
                         device="cuda")
        t_str = med(lambda: sm.strassen_mm(A32, B32, Cw, 1, sm.CLASSIC, sm.PREC_BF16X3, workspace=ws))
        rows.append({"m": m, "n": n, "k": k, "bf16_ms": t_bf16, "bf16_split_k": split_bf16,
                     "strassen_d1_bf16x3_ms": t_str, "strassen_faster": t_str < t_bf16})
        del ws, A32, B32, Cw
    return rows
