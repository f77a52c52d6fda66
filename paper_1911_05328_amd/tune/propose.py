"""Schedule proposal for one (shape, dtype, workspace budget): the cost
model's argmin over the feasible schedules, optionally refined by timing the
model's top-k candidates; exhaustive timing is the fallback and the arbiter."""
from __future__ import annotations

import numpy as np

import paper_1911_05328_amd as sm

from . import space
from .dataset import DEFAULT_IDX


def feasible(dtype, m, n, k, budget, accurate=None):
    """Schedules the planner runs within the budget: an fp32 schedule without
    Strassen counts when either its pre-split-plane or its in-kernel-split
    variant fits, as in the training samples.  accurate: the model's
    (3 x NSCHED) accuracy mask; masked schedules are not feasible."""
    out = []
    for j in range(space.NSCHED):
        if accurate is not None and not accurate[space.DTYPES.index(dtype)][j]:
            out.append(False)
            continue
        ok = False
        for ik in ((False, True) if space.has_inkernel_variant(dtype, j) else (False,)):
            w = space.workspace_bytes(dtype, m, n, k, j, inkernel=ik)
            ok = ok or (w is not None and w <= budget)
        out.append(ok)
    return np.array(out, dtype=bool)


def propose(model, m, n, k, dtype, budget, topk: int = 1, timer=None) -> int:
    """Index into space.SCHEDULES."""
    feas = feasible(dtype, m, n, k, budget, getattr(model, "accurate", None))
    pred = model.predict(np.array([space.features(m, n, k, dtype, budget)]))[0]
    pred = np.where(feas, pred, np.inf)
    order = np.argsort(pred)
    if topk <= 1 or timer is None:
        return int(order[0])
    cand = [int(j) for j in order[:topk] if np.isfinite(pred[j])]
    times = [timer.time(dtype, m, n, k, j) for j in cand]
    return cand[int(np.argmin(times))]


def exhaustive(timer, m, n, k, dtype, budget) -> int:
    feas = feasible(dtype, m, n, k, budget)
    best, arg = np.inf, DEFAULT_IDX
    for j in np.flatnonzero(feas):
        t = timer.time(dtype, m, n, k, int(j))
        if t is not None and t < best:
            best, arg = t, int(j)
    return arg


def heuristic(m, n, k, dtype, budget, feas_row) -> int:
    """The library's own planner (no model): its tile / k-split for this
    budget mapped into the space; the default schedule when that choice is not
    a timed, feasible schedule (e.g. atomic merging of (min,+) splits)."""
    sr, dt = space.semiring_and_dtype(dtype)
    prec = space.precision(dtype, 0)
    st, p = sm.plan(sr, dt, m, n, k, int(budget), sm.make_schedule(precision=prec))
    if st != sm.MM_OK or p["tar_levels"] > 0 or p["bands"] > 1:
        return DEFAULT_IDX
    key = (0, int(p["sched"]["split_k"]), int(p["sched"]["tile"]))
    if key not in space.SCHEDULES:
        return DEFAULT_IDX
    j = space.SCHEDULES.index(key)
    return j if feas_row[j] else DEFAULT_IDX


def roofline_time(m, n, k, dtype, idx, cus=256):
    """Analytic roofline estimate (seconds) of schedule idx, no measurement:
    executed work over the datasheet rate, scaled by the fraction of CUs the
    grid fills and a per-tile-size efficiency, against the bytes the
    schedule moves over 8 TB/s, plus 5 us per launch."""
    d, s, t = space.SCHEDULES[idx]
    lm, ln, lk = (-(-x // 2 ** d) for x in (m, n, k))
    leaves = 7 ** d
    wgs = -(-lm // t) * -(-ln // t) * s * leaves
    fill = min(1.0, wgs / cus)
    if dtype == "i32":
        rate = 78.6e12 * {32: 0.5, 64: 0.75, 128: 1.0, 256: 1.0}[t]  # lane-ops/s
        work = 1.5 * lm * ln * lk * leaves
        elt = 4
    else:
        rate = 2.5e15 * {32: 0.2, 64: 0.4, 128: 0.7, 256: 1.0}[t]  # bf16 MFMA flop/s
        work = 2.0 * lm * ln * lk * leaves * (3 if dtype == "f32" else 1)
        elt = 4 if dtype == "f32" else 2
    compute = work / (rate * fill)
    # operands re-read once per tile row / column, C and the k-split
    # temporaries read and written, Strassen operands formed and read back
    nbytes = (lm * lk * elt * -(-ln // t) + lk * ln * elt * -(-lm // t)) * leaves / 8.0  # L2 reuse ~8x
    nbytes += 8.0 * m * n + 8.0 * (s - 1) * lm * ln * leaves
    if d > 0:
        g = (7.0 / 4.0) ** d
        nbytes += 4.0 * (m * k + k * n) * (1 + g) + 4.0 * m * n * (g + 2)
    launches = 1 + (1 if s > 1 else 0) + (3 if d > 0 else 0)
    return max(compute, nbytes / 8e12) + 5e-6 * launches


def roofline_heuristic(m, n, k, dtype, feas_row) -> int:
    """The feasible schedule of least analytic roofline time."""
    best, arg = float("inf"), DEFAULT_IDX
    for j in range(space.NSCHED):
        if feas_row[j]:
            tj = roofline_time(m, n, k, dtype, j)
            if tj < best:
                best, arg = tj, j
    return arg

