"""Training / evaluation samples for the cost model from the timing DB.

Each DB row (one shape and dtype, every schedule timed) yields several
samples, one per workspace budget drawn log-uniformly in [1/8, 8] x |C|
bytes; a schedule is feasible for a sample when it is supported for the
dtype, its workspace fits the budget and its measured error is within the
target (fp32 schedules).  As in the planner, an fp32
schedule without Strassen uses pre-split bf16 planes when they fit the
budget and splits inside the tile kernel otherwise, so its time for a
budget is the one of the variant the planner would run.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import space

DB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "timings_mi355x.jsonl")
DEFAULT_IDX = space.SCHEDULES.index((0, 1, 128))  # no Strassen, no split, largest tile


def load_db(path=DB_PATH):
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def within_target(r, j, max_error=space.TARGET_ERROR) -> bool:
    """Schedule j of DB row r meets the error target (rows without recorded
    errors, and dtypes whose products are exact up to fp32 accumulation,
    record None: accepted)."""
    errs = r.get("errors")
    if errs is None or errs[j] is None:
        return True
    return errs[j] <= max_error


def accuracy_mask(rows, max_error=space.TARGET_ERROR):
    """(3 x NSCHED) 0/1 per space dtype: 1 when every measured error of the
    schedule over `rows` is within the target."""
    mask = np.ones((len(space.DTYPES), space.NSCHED))
    for r in rows:
        d = space.DTYPES.index(r["dtype"])
        for j in range(space.NSCHED):
            if not within_target(r, j, max_error):
                mask[d, j] = 0.0
    return mask


def samples(rows, budgets_per_row=4, seed=1911, max_error=space.TARGET_ERROR):
    """Returns X (N x 7), logT (N x NSCHED; 0 where unmeasured), feasible mask
    (N x NSCHED), times (N x NSCHED, inf where infeasible), meta [(row index,
    budget)].  A schedule measured above `max_error` on a row is not
    feasible for it (None: errors ignored)."""
    g = np.random.Generator(np.random.PCG64(seed))
    X, T, F, TT, meta = [], [], [], [], []
    for ri, r in enumerate(rows):
        cbytes = r["m"] * r["n"] * space.c_elem_bytes(r["dtype"])
        ik_t = r.get("times_inkernel_ms") or [None] * space.NSCHED
        ik_w = r.get("ws_inkernel_bytes") or [None] * space.NSCHED
        for _ in range(budgets_per_row):
            budget = cbytes * 2.0 ** g.uniform(-3.0, 3.0)
            t, feas = np.full(space.NSCHED, np.inf), np.zeros(space.NSCHED, dtype=bool)
            for j in range(space.NSCHED):
                if max_error is not None and not within_target(r, j, max_error):
                    continue
                for tj, wj in ((r["times_ms"][j], r["ws_bytes"][j]), (ik_t[j], ik_w[j])):
                    if tj is not None and wj is not None and wj <= budget:
                        t[j], feas[j] = tj, True
                        break
            X.append(space.features(r["m"], r["n"], r["k"], r["dtype"], budget))
            T.append(np.where(feas, np.log(np.where(np.isfinite(t), t, 1.0)), 0.0))
            F.append(feas)
            TT.append(np.where(feas, t, np.inf))
            meta.append((ri, budget))
    return (np.array(X), np.array(T), np.array(F, dtype=np.float64), np.array(TT), meta)


def regret(pick, times):
    """t(pick) / t(best feasible) - 1 per sample."""
    best = times.min(axis=1)
    return times[np.arange(len(pick)), pick] / best - 1.0


def summary(r):
    return {"mean": float(np.mean(r)), "median": float(np.median(r)), "p90": float(np.percentile(r, 90)),
            "max": float(np.max(r))}
