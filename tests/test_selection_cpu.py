"""Schedule selection for calls without a schedule (host code, no GPU):
the library's own evaluation of the trained cost model and its lookup of
measured timings, against the same computations written out in numpy over
the tuner's schedule space and feasibility rule.

Pins: the proposal is the argmin of the network's outputs over the schedules
the planner accepts within the budget and the model's accuracy mask keeps,
and its predicted time is the exp of
that output; a timing lookup is the least measured time among the entries
that fit; mm_plan without a schedule follows timings, then the model, then
the built-in planner, and comes back to the built-in planner once cleared."""
import math

import numpy as np
import pytest

import paper_1911_05328_amd as sm
from paper_1911_05328_amd import _lib
from paper_1911_05328_amd.tune import dataset, propose, selection, space


@pytest.fixture
def clean():
    sm.selection_clear()
    yield
    sm.selection_clear()


def numpy_predict(z, x):
    h = np.asarray(x, np.float64)
    for l in range(4):
        h = z[f"W{l}"].astype(np.float64) @ h + z[f"b{l}"].astype(np.float64)
        if l < 3:
            h = np.maximum(h, 0.0)
    # the ABI takes every parameter as float, the standardisation included
    return h * float(np.float32(z["t_std"])) + float(np.float32(z["t_mean"]))


def cases(seed, count):
    g = np.random.default_rng(seed)
    out = []
    for i in range(count):
        dtype = space.DTYPES[i % 3]
        m, n, k = (int(2 ** g.uniform(7, 14)) for _ in range(3))
        budget = int(m * n * 4 * 2.0 ** g.uniform(-3, 3))
        out.append((dtype, m, n, k, budget))
    return out


def key(s):
    d = s.as_dict() if not isinstance(s, dict) else s
    return (d["strassen_depth"], d["split_k"], d["tile"])


def test_param_count_and_bad_loads(clean):
    L = _lib.lib()
    assert L.mm_cost_model_param_count() == 2 + (7 * 64 + 64) + 2 * (64 * 64 + 64) + (64 * 64 + 64) + 3 * 64
    p = selection.model_params()
    with pytest.raises(sm.StarmmError):
        sm.cost_model_load(p[:-1])
    q = p.copy()
    q[1] = 0.0  # t_std must be positive
    with pytest.raises(sm.StarmmError):
        sm.cost_model_load(q)
    q = p.copy()
    q[100] = np.nan
    with pytest.raises(sm.StarmmError):
        sm.cost_model_load(q)
    q = p.copy()
    q[-1] = 0.5  # accuracy mask entries are 0 or 1
    with pytest.raises(sm.StarmmError):
        sm.cost_model_load(q)
    st, s, _ = sm.propose_schedule(sm.PLUS_TIMES, sm.DT_F32, 256, 256, 256, 1 << 20)
    assert st == sm.MM_ERR_UNSUPPORTED and s is None  # nothing was loaded
    # a timing whose schedule the planner rejects for its problem
    bad = (sm.MIN_PLUS, sm.DT_I32, 64, 64, 64, sm.make_schedule(tile=256, split_k=1), 1.0)
    good = (sm.MIN_PLUS, sm.DT_I32, 64, 64, 64, sm.make_schedule(tile=64, split_k=1), 1.0)
    with pytest.raises(sm.StarmmError):
        sm.tuned_load([good, bad])
    assert sm.tuned_lookup(sm.MIN_PLUS, sm.DT_I32, 64, 64, 64, 1 << 30)[0] == sm.MM_ERR_UNSUPPORTED
    with pytest.raises(sm.StarmmError):
        sm.tuned_load([(sm.MIN_PLUS, sm.DT_I32, 64, 64, 64, sm.make_schedule(tile=64), -1.0)])


def test_proposal_is_masked_argmin_of_the_network(clean):
    z = np.load(selection.MODEL_PATH)
    sm.cost_model_load(selection.model_params())
    for dtype, m, n, k, budget in cases(7, 45):
        sr, dt = space.semiring_and_dtype(dtype)
        pred = numpy_predict(z, space.features(m, n, k, dtype, budget))
        feas = propose.feasible(dtype, m, n, k, budget, selection.accuracy_mask())
        assert feas.any()
        want = int(np.argmin(np.where(feas, pred, np.inf)))
        st, s, ms = sm.propose_schedule(sr, dt, m, n, k, budget)
        assert st == sm.MM_OK
        got = space.SCHEDULES.index(key(s))
        assert feas[got]
        # equal up to float rounding of near ties
        assert got == want or abs(pred[got] - pred[want]) < 1e-9, (dtype, m, n, k, budget, got, want)
        assert math.isclose(ms, math.exp(pred[got]), rel_tol=1e-9)
        assert s.as_dict() == space.schedule(dtype, m, got).as_dict()
        # a call without a schedule plans exactly the proposal
        st, p = sm.plan(sr, dt, m, n, k, budget)
        assert st == sm.MM_OK and key(p["sched"]) == key(s) and p["ws_bytes"] <= budget
    # pairs outside the model's space: no proposal, the planner decides
    st, s, _ = sm.propose_schedule(sm.MAX_PLUS, sm.DT_I32, 300, 300, 300, 1 << 30)
    assert st == sm.MM_ERR_UNSUPPORTED
    sm.selection_clear()
    ref = sm.plan(sm.MAX_PLUS, sm.DT_I32, 300, 300, 300, 1 << 30)
    sm.cost_model_load(selection.model_params())
    assert sm.plan(sm.MAX_PLUS, sm.DT_I32, 300, 300, 300, 1 << 30) == ref


def test_timings_lookup_and_precedence(clean):
    rows = dataset.load_db()
    g = np.random.default_rng(11)
    picked = [rows[int(i)] for i in g.choice(len(rows), 24, replace=False)]
    sm.tuned_load(selection.timing_entries(picked))
    for r in picked:
        dtype, m, n, k = r["dtype"], r["m"], r["n"], r["k"]
        sr, dt = space.semiring_and_dtype(dtype)
        for budget in (int(m * n * 4 * 2.0 ** e) for e in (-3, 0, 3)):
            best, arg = np.inf, None
            ik = r.get("times_inkernel_ms") or [None] * space.NSCHED
            for j in range(space.NSCHED):
                if not dataset.within_target(r, j):
                    continue  # measured above the error target: not loaded
                for t, inkernel in ((r["times_ms"][j], False), (ik[j], True)):
                    w = space.workspace_bytes(dtype, m, n, k, j, inkernel=inkernel) if t is not None else None
                    if w is not None and w <= budget and t < best:
                        best, arg = t, (j, inkernel)
            st, s, ms = sm.tuned_lookup(sr, dt, m, n, k, budget)
            if arg is None:
                assert st == sm.MM_ERR_UNSUPPORTED
                continue
            assert st == sm.MM_OK and ms == best
            assert s.as_dict() == space.schedule(dtype, m, arg[0], inkernel=arg[1]).as_dict()
            stp, p = sm.plan(sr, dt, m, n, k, budget)
            assert stp == sm.MM_OK and key(p["sched"]) == key(s)
    # with the model loaded too, a timed shape keeps its timing and an untimed one gets the proposal
    sm.cost_model_load(selection.model_params())
    r = picked[0]
    sr, dt = space.semiring_and_dtype(r["dtype"])
    budget = r["m"] * r["n"] * 4
    _, s_db, _ = sm.tuned_lookup(sr, dt, r["m"], r["n"], r["k"], budget)
    assert key(sm.plan(sr, dt, r["m"], r["n"], r["k"], budget)[1]["sched"]) == key(s_db)
    m2 = r["m"] + 1
    _, s_mlp, _ = sm.propose_schedule(sr, dt, m2, r["n"], r["k"], budget)
    assert key(sm.plan(sr, dt, m2, r["n"], r["k"], budget)[1]["sched"]) == key(s_mlp)


def test_clear_restores_the_builtin_planner(clean):
    probs = [(sm.PLUS_TIMES, sm.DT_F32, 1000, 3000, 2000, 1 << 26), (sm.MIN_PLUS, sm.DT_I32, 700, 700, 5000, 1 << 22),
             (sm.PLUS_TIMES, sm.DT_BF16, 4096, 4096, 512, 1 << 28)]
    before = [sm.plan(*p) for p in probs]
    sm.cost_model_load(selection.model_params())
    assert any(sm.plan(*p) != b for p, b in zip(probs, before))
    sm.selection_clear()
    assert [sm.plan(*p) for p in probs] == before
