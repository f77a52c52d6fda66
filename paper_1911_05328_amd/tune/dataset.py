"""Training / evaluation samples for the cost model from the timing DB.

Each DB row (one shape and dtype, every schedule timed) yields several
samples, one per workspace budget drawn log-uniformly in [1/8, 8] x |C|
bytes; a schedule is feasible for a sample when it is supported for the
dtype and its workspace fits the budget.
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


def samples(rows, budgets_per_row=4, seed=1911):
    """Returns X (N x 7), logT (N x 48; 0 where unmeasured), feasible mask
    (N x 48), times (N x 48, inf where infeasible), meta [(row index, budget)]."""
    g = np.random.Generator(np.random.PCG64(seed))
    X, T, F, TT, meta = [], [], [], [], []
    for ri, r in enumerate(rows):
        cbytes = r["m"] * r["n"] * space.c_elem_bytes(r["dtype"])
        for _ in range(budgets_per_row):
            budget = cbytes * 2.0 ** g.uniform(-3.0, 3.0)
            feas = np.array([t is not None and w is not None and w <= budget
                             for t, w in zip(r["times_ms"], r["ws_bytes"])], dtype=bool)
            t = np.array([x if x is not None else np.inf for x in r["times_ms"]], dtype=np.float64)
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
