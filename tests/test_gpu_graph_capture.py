"""GPU: a product's launch sequence can be captured in a HIP graph and
replayed (it enqueues kernels only: no allocation, no memset, no host
synchronisation).  Each replay, with eager work between replays, gives the
bits of the same call made eagerly: the Strassen step (pre-additions into
planes, leaf products, post-additions), a (min,+) product whose k-split
merges through temporaries, and a BF16x3 product over pre-split planes."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402


def check_capture(call, C, C0):
    C.copy_(C0)
    call()
    torch.cuda.synchronize()
    want = C.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        C.copy_(C0)
        call()  # warm on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        call()
    for rep in range(3):
        C.copy_(C0)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C.view(torch.int32), want.view(torch.int32)), rep
    del g


def test_strassen_step_replays_bitwise():
    sm.profile_enable(False)
    n = 1536
    A = torch.from_numpy(si.normal_f32(1, (n, n))).cuda()
    B = torch.from_numpy(si.normal_f32(2, (n, n))).cuda()
    C0 = torch.from_numpy(si.normal_f32(3, (n, n))).cuda()
    C = torch.empty_like(C0)
    ws = torch.empty(sm.strassen_workspace_bytes(n, n, n, 1, sm.CLASSIC, sm.PREC_BF16X3), dtype=torch.uint8,
                     device="cuda")
    check_capture(lambda: sm.strassen_mm(A, B, C, 1, sm.CLASSIC, sm.PREC_BF16X3, workspace=ws), C, C0)


def test_minplus_split_temporaries_replay_bitwise():
    m, n, k = 700, 530, 2100
    A = torch.from_numpy(si.semiring_operand(sm.MIN_PLUS, 4, (m, k))).cuda()
    B = torch.from_numpy(si.semiring_operand(sm.MIN_PLUS, 5, (k, n))).cuda()
    C0 = torch.from_numpy(si.semiring_operand(sm.MIN_PLUS, 6, (m, n))).cuda()
    C = torch.empty_like(C0)
    ws = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    sched = sm.make_schedule(tile=64, split_k=4, band_rows=128)
    check_capture(lambda: sm.semiring_mm(A, B, C, sm.MIN_PLUS, workspace=ws, schedule=sched), C, C0)


def test_bf16x3_planes_replay_bitwise():
    m, n, k = 900, 1100, 1300
    A = torch.from_numpy(si.normal_f32(7, (m, k))).cuda()
    B = torch.from_numpy(si.normal_f32(8, (k, n))).cuda()
    C0 = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    C = torch.empty_like(C0)
    sched = sm.make_schedule(tile=256, split_k=2, precision=sm.PREC_BF16X3, band_rows=m)
    ws = torch.empty(sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, sched), dtype=torch.uint8, device="cuda")
    check_capture(lambda: sm.semiring_mm(A, B, C, sm.PLUS_TIMES, workspace=ws, schedule=sched), C, C0)
