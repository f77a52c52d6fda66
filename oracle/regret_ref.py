"""Oracle for judging a schedule proposal: exhaustive search and regret.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Not from the paper: the
learned schedule proposal is judged against exhaustive tuning, which times
every schedule of the space and keeps the fastest one that runs within the
workspace budget.  Written out from that definition with plain loops:

  feasible(j)   schedule j has a measured time and its workspace need is at
                most the budget; where a schedule has two timed variants (an
                fp32 product over pre-split planes, and the same schedule
                splitting inside the kernel), the first variant that fits is
                the one that runs, as the planner chooses
  best          the feasible j of least time (ties: the lowest index)
  regret(pick)  t(pick) / t(best) - 1, >= 0 for every feasible pick, 0 for best
  acceptable(j) additionally, when an error bound is given, the measured
                relative error of schedule j does not exceed it
"""
from __future__ import annotations

import math


def run_time(variants, budget):
    """Time of the variant that runs under `budget`: the first (time, ws)
    pair, in the order given, whose time is measured and whose workspace
    fits; None when none fits."""
    for t, ws in variants:
        if t is None or ws is None:
            continue
        if ws <= budget:
            return float(t)
    return None


def exhaustive_best(times, budget, errors=None, max_error=None):
    """Index and time of the fastest feasible schedule.

    times[j]  -- list of (time_ms, workspace_bytes) variants of schedule j
    budget    -- workspace bytes available
    errors[j] -- measured relative error of schedule j (None: unmeasured)
    max_error -- when given, schedules whose error is unmeasured or above it
                 are not feasible
    Returns (index, time) or (None, None) when nothing is feasible."""
    best_j, best_t = None, None
    for j in range(len(times)):
        t = run_time(times[j], budget)
        if t is None:
            continue
        if max_error is not None:
            e = None if errors is None else errors[j]
            if e is None or not (e <= max_error):
                continue
        if best_t is None or t < best_t:
            best_j, best_t = j, t
    return best_j, best_t


def regret(t_pick, t_best):
    """t(pick) / t(best) - 1."""
    if t_best is None or t_pick is None or not math.isfinite(t_pick):
        return math.inf
    return t_pick / t_best - 1.0
