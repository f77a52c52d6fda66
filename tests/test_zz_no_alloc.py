"""mm_semiring_static (the entry point that allocates nothing: its workspace
is the library's static scratch array) against mm_semiring with a caller
workspace, same schedules, on the GPU through the C ABI.  Two calls in a row,
the second on a smaller input, so the second reads scratch the first left
behind."""
import numpy as np
import pytest
import torch

import paper_1911_05328_amd as sm
import synth_inputs as si

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _pair(semiring, A, B, C0, sched, ws_bytes):
    """(C from mm_semiring with a caller workspace, C from mm_semiring_static)."""
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
    C1 = _dev(C0)
    sm.semiring_mm(_dev(A), _dev(B), C1, semiring, workspace=ws, schedule=sched)
    C2 = _dev(C0)
    sm.semiring_mm_static(_dev(A), _dev(B), C2, semiring, schedule=sched)
    torch.cuda.synchronize()
    return C1.cpu().numpy(), C2.cpu().numpy()


@pytest.mark.parametrize("shapes", [((700, 900, 1500), (300, 200, 500))])
def test_static_minplus_split_matches_workspace_entry(shapes):
    # k split into 4 (three temporaries in the scratch), then 2
    for i, ((m, n, k), split) in enumerate(zip(shapes, (4, 2))):
        print(f"static (min,+) call {i}: {m}x{n}x{k} split {split}", flush=True)
        A = si.minplus_i32(11 + i, (m, k))
        B = si.minplus_i32(21 + i, (k, n))
        C0 = si.semiring_init(sm.MIN_PLUS, (m, n))
        sched = sm.make_schedule(tile=64, split_k=split)
        ws = sm.workspace_bytes(sm.MIN_PLUS, sm.DT_I32, m, n, k, sched)
        assert 0 < ws <= sm.STATIC_SCRATCH_BYTES
        ref, got = _pair(sm.MIN_PLUS, A, B, C0, sched, ws)
        assert np.array_equal(ref, got)


def test_static_bf16x3_planes_match_workspace_entry():
    # fp32 through BF16x3 planes (the split operands live in the scratch),
    # 2-way k-split merged in fixed order: both entries give the same bits
    for i, (m, n, k) in enumerate(((1000, 777, 1200), (260, 130, 333))):
        print(f"static BF16x3 call {i}: {m}x{n}x{k}", flush=True)
        A = si.uniform_f32(31 + i, (m, k))
        B = si.uniform_f32(41 + i, (k, n))
        C0 = si.uniform_f32(51 + i, (m, n))
        sched = sm.make_schedule(tile=128, split_k=2, precision=sm.PREC_BF16X3)
        ws = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, sched)
        assert ws <= sm.STATIC_SCRATCH_BYTES
        st, info = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, sm.STATIC_SCRATCH_BYTES, sched)
        assert st == sm.MM_OK and info["ws_bytes"] == ws
        ref, got = _pair(sm.PLUS_TIMES, A, B, C0, sched, ws)
        assert np.array_equal(ref, got)


def test_static_planner_choice_matches_workspace_entry():
    # no schedule: the built-in planner under the scratch budget, against
    # mm_semiring given a workspace of the same size
    for i, (m, n, k) in enumerate(((512, 640, 3000), (100, 90, 80))):
        print(f"static planner call {i}: {m}x{n}x{k}", flush=True)
        A = si.minplus_i32(61 + i, (m, k))
        B = si.minplus_i32(71 + i, (k, n))
        C0 = si.semiring_init(sm.MIN_PLUS, (m, n))
        ref, got = _pair(sm.MIN_PLUS, A, B, C0, None, sm.STATIC_SCRATCH_BYTES)
        assert np.array_equal(ref, got)


def test_static_schedule_beyond_scratch_is_refused():
    n = 4096
    A = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    C = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    with pytest.raises(sm.StarmmError) as e:
        sm.semiring_mm_static(A, A, C, sm.MIN_PLUS, schedule=sm.make_schedule(tile=128, split_k=8, band_rows=n))
    assert e.value.status == sm.MM_ERR_WORKSPACE
