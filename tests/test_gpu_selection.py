"""Calls without a schedule once the tuner's results are loaded (GPU).

* The library's host evaluation of the cost model proposes the schedule the
  trained model proposes when evaluated by the library's own MLP kernels.
* mm_semiring without a schedule runs the selected schedule: its result is
  bit for bit that of the same schedule passed explicitly, within that
  schedule's error bound against the float64 oracle ((+,x)), and exact
  against the oracle ((min,+)); a loaded timing for the exact shape wins
  over the model; after clearing, the built-in planner decides again.
"""
import math

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402
from paper_1911_05328_amd.tune import propose, selection, space  # noqa: E402
from paper_1911_05328_amd.tune.mlp import CostModel  # noqa: E402


@pytest.fixture
def clean():
    sm.selection_clear()
    yield
    sm.selection_clear()


def key(d):
    return (d["strassen_depth"], d["split_k"], d["tile"])


def test_library_proposal_matches_model_on_gpu(clean):
    model = CostModel.load(selection.MODEL_PATH)
    sm.cost_model_load(selection.model_params())
    g = np.random.default_rng(21)
    for i in range(36):
        dtype = space.DTYPES[i % 3]
        m, n, k = (int(2 ** g.uniform(7, 14)) for _ in range(3))
        budget = int(m * n * 4 * 2.0 ** g.uniform(-3, 3))
        sr, dt = space.semiring_and_dtype(dtype)
        want = propose.propose(model, m, n, k, dtype, budget)
        pred = model.predict(np.array([space.features(m, n, k, dtype, budget)]))[0]
        st, s, ms = sm.propose_schedule(sr, dt, m, n, k, budget)
        assert st == sm.MM_OK
        got = space.SCHEDULES.index(key(s.as_dict()))
        # fp32 kernels against double host arithmetic: equal but for near ties
        assert got == want or abs(pred[got] - pred[want]) < 1e-4, (dtype, m, n, k, budget)
        assert abs(math.log(ms) - pred[got]) < 1e-4


def test_null_schedule_f32_runs_the_proposal(clean):
    m, n, k = 1500, 1301, 1700
    A = si.normal_f32(si.BASE_SEED + 40, (m, k))
    B = si.normal_f32(si.BASE_SEED + 41, (k, n))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = oracle.fp64_ref(A, B)
    sm.cost_model_load(selection.model_params())
    for budget in (m * n * 4 // 8, m * n * 4, m * n * 4 * 8):
        st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, budget)
        assert st == sm.MM_OK and p["ws_bytes"] <= budget
        s = p["sched"]
        ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
        C1 = torch.zeros((m, n), dtype=torch.float32, device="cuda")
        sm.semiring_mm(dA, dB, C1, sm.PLUS_TIMES, workspace=ws)
        explicit = sm.make_schedule(tile=s["tile"], split_k=s["split_k"], strassen_depth=s["strassen_depth"],
                                    variant=s["variant"], precision=s["precision"],
                                    band_rows=s["band_rows"] if s["strassen_depth"] == 0 else 0,
                                    strassen_layout=s["strassen_layout"])
        C2 = torch.zeros((m, n), dtype=torch.float32, device="cuda")
        sm.semiring_mm(dA, dB, C2, sm.PLUS_TIMES, workspace=ws, schedule=explicit)
        torch.cuda.synchronize()
        got = C1.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), C2.cpu().numpy().view(np.uint32)), (budget, s)
        # the space's fp32 schedules are held to the error target
        assert oracle.rel_fro(got, ref) <= space.TARGET_ERROR, (budget, s)


def test_proposed_fp32_schedules_meet_the_error_target_on_held_out_shapes(clean):
    # The model's accuracy mask comes from the training shapes' measured
    # errors; on held-out fp32 shapes (up to 4096 in each dimension here) at
    # three budgets, every proposed schedule's result stays within 1e-5 of
    # the oracle's float64 product (sampled rows).
    from paper_1911_05328_amd.tune import dataset
    rows = [r for r in dataset.load_db() if r["split"] == "test" and r["dtype"] == "f32"
            and max(r["m"], r["n"], r["k"]) <= 4096][:12]
    assert len(rows) >= 8
    sm.cost_model_load(selection.model_params())
    for r in rows:
        m, n, k = r["m"], r["n"], r["k"]
        A = si.normal_f32(m + 7 * n, (m, k))
        B = si.normal_f32(k + 7 * n, (k, n))
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        rws = np.unique(np.linspace(0, m - 1, 24).round().astype(np.int64))
        ref = oracle.fp64_rows(A, B, rws)
        for budget in (m * n * 4 // 8, m * n * 4, m * n * 4 * 8):
            st, s, _ = sm.propose_schedule(sm.PLUS_TIMES, sm.DT_F32, m, n, k, budget)
            assert st == sm.MM_OK
            ws = torch.empty(max(budget, 1), dtype=torch.uint8, device="cuda")
            C = torch.zeros((m, n), dtype=torch.float32, device="cuda")
            sm.semiring_mm(dA, dB, C, sm.PLUS_TIMES, workspace=ws, schedule=s)
            torch.cuda.synchronize()
            err = oracle.rel_fro(C.cpu().numpy()[rws], ref)
            assert err <= space.TARGET_ERROR, (m, n, k, budget, s.as_dict(), err)


def test_null_schedule_minplus_timing_wins_then_clear(clean):
    m, n, k = 700, 515, 900
    A = si.semiring_operand(sm.MIN_PLUS, si.BASE_SEED + 50, (m, k))
    B = si.semiring_operand(sm.MIN_PLUS, si.BASE_SEED + 51, (k, n))
    C0 = si.semiring_operand(sm.MIN_PLUS, si.BASE_SEED + 52, (m, n))
    ref = oracle.brute(oracle.MIN_PLUS, A, B, C0)
    fast = sm.make_schedule(tile=32, split_k=4, band_rows=m)
    slow = sm.make_schedule(tile=64, split_k=1, band_rows=m)
    budget = 1 << 24
    builtin = sm.plan(sm.MIN_PLUS, sm.DT_I32, m, n, k, budget)[1]["sched"]
    sm.cost_model_load(selection.model_params())
    sm.tuned_load([(sm.MIN_PLUS, sm.DT_I32, m, n, k, slow, 2.0), (sm.MIN_PLUS, sm.DT_I32, m, n, k, fast, 1.0)])
    for phase in ("timed", "cleared"):
        st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, m, n, k, budget)
        assert st == sm.MM_OK
        if phase == "timed":
            assert (p["sched"]["tile"], p["sched"]["split_k"]) == (32, 4)
        else:
            assert p["sched"] == builtin
        ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
        dC = torch.from_numpy(np.ascontiguousarray(C0, np.int32)).cuda()
        sm.semiring_mm(torch.from_numpy(np.ascontiguousarray(A, np.int32)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(B, np.int32)).cuda(), dC, sm.MIN_PLUS, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), phase
        sm.selection_clear()
