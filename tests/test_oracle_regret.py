"""Pins the regret oracle (exhaustive search over timed schedules) to brute
force on small tables, then checks the tuner's sample builder and regret
against it on the committed timing database.  CPU only."""
import itertools
import math

import numpy as np
import pytest

from oracle import regret_ref as rr


def _all_orders_best(times, budget):
    """Brute force: the feasible index whose time no other feasible time
    undercuts (lowest index among equals)."""
    feas = []
    for j, variants in enumerate(times):
        t = None
        for tv, wv in variants:
            if tv is not None and wv is not None and wv <= budget:
                t = tv
                break
        if t is not None:
            feas.append((j, t))
    for j, t in feas:
        if all(t < u or (t == u and j <= i) for i, u in feas):
            return j, t
    return None, None


def test_exhaustive_best_brute_force_small_tables():
    g = np.random.default_rng(9)
    for _ in range(300):
        ns = int(g.integers(1, 7))
        times = []
        for _j in range(ns):
            nv = int(g.integers(1, 3))
            var = []
            for _v in range(nv):
                t = None if g.random() < 0.2 else float(g.integers(1, 6))  # ties are common
                w = None if g.random() < 0.1 else int(g.integers(0, 100))
                var.append((t, w))
            times.append(var)
        budget = int(g.integers(0, 120))
        assert rr.exhaustive_best(times, budget) == _all_orders_best(times, budget)


def test_regret_definition():
    times = [[(4.0, 0)], [(2.0, 50)], [(3.0, 10)], [(1.0, 500)]]
    j, t = rr.exhaustive_best(times, 60)
    assert (j, t) == (1, 2.0)  # schedule 3 needs more than the budget
    assert rr.regret(t, t) == 0.0
    assert rr.regret(4.0, t) == pytest.approx(1.0)
    assert rr.regret(3.0, t) == pytest.approx(0.5)
    assert rr.exhaustive_best(times, 1000) == (3, 1.0)
    assert rr.exhaustive_best(times, -1) == (None, None)
    # variant order: the first variant that fits runs (planes before in-kernel)
    assert rr.exhaustive_best([[(5.0, 100), (7.0, 0)]], 100) == (0, 5.0)
    assert rr.exhaustive_best([[(5.0, 100), (7.0, 0)]], 99) == (0, 7.0)


def test_error_bound_masks_schedules():
    times = [[(1.0, 0)], [(2.0, 0)], [(3.0, 0)]]
    assert rr.exhaustive_best(times, 0, errors=[2e-5, 9e-6, 1e-6], max_error=1e-5) == (1, 2.0)
    assert rr.exhaustive_best(times, 0, errors=[2e-5, None, 1e-6], max_error=1e-5) == (2, 3.0)
    assert rr.exhaustive_best(times, 0, errors=[2e-5, 3e-5, 4e-5], max_error=1e-5) == (None, None)
    assert rr.exhaustive_best(times, 0, errors=[2e-5, 3e-5, 4e-5]) == (0, 1.0)  # no bound given


def test_tuner_samples_and_regret_match_the_oracle():
    from paper_1911_05328_amd.tune import dataset, space

    rows = dataset.load_db()[:120]
    X, logT, F, TT, meta = dataset.samples(rows, budgets_per_row=3, seed=7)
    g = np.random.default_rng(3)
    picks = []
    for si, (ri, budget) in enumerate(meta):
        r = rows[ri]
        ik_t = r.get("times_inkernel_ms") or [None] * space.NSCHED
        ik_w = r.get("ws_inkernel_bytes") or [None] * space.NSCHED
        table = [[(r["times_ms"][j], r["ws_bytes"][j]), (ik_t[j], ik_w[j])] for j in range(space.NSCHED)]
        # fp32 schedules carry measured errors and must meet the target;
        # bf16 / (min,+) products record none
        errs = r.get("errors") if r["dtype"] == "f32" else None
        bound = space.TARGET_ERROR if errs is not None else None
        j, t = rr.exhaustive_best(table, budget, errors=errs, max_error=bound)
        assert j is not None
        assert TT[si].min() == t
        # the tuner's feasibility mask is the oracle's
        for jj in range(space.NSCHED):
            ok = rr.run_time(table[jj], budget) is not None
            if bound is not None:
                ok = ok and errs[jj] is not None and errs[jj] <= bound
            assert bool(F[si, jj]) == ok
        feas = [jj for jj in range(space.NSCHED) if F[si, jj]]
        picks.append((int(g.choice(feas)), table, budget, t))
    assert len(picks) == len(meta)
    pick_idx = np.array([p[0] for p in picks])
    got = dataset.regret(pick_idx, TT)
    want = np.array([rr.regret(rr.run_time(tab[p], b), t) for p, tab, b, t in picks])
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    # exhaustive search has no regret
    best_idx = np.argmin(TT, axis=1)
    assert np.all(dataset.regret(best_idx, TT) == 0.0)
    assert math.isinf(rr.regret(None, 1.0))
