"""Empty products through every entry point, on real (empty) device tensors:
with k = 0 the sum over l in eq. mm-dac is empty, so C keeps its values (the
semiring zero is neutral under its (+)); with m = 0 or n = 0 there is no
output.  Explicit k-splits, Strassen levels and FP16x3 need no workspace
for them, and a batch mixes empty problems with ordinary ones."""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

SHAPES = [(70, 90, 0), (0, 90, 40), (70, 0, 40), (0, 0, 0)]


def _c0(m, n, dtype):
    if dtype == torch.int32:
        return torch.from_numpy(si.minplus_i32(5, (m, n))).cuda()
    return torch.from_numpy(si.normal_f32(5, (m, n))).cuda()


@pytest.mark.parametrize("shape", SHAPES)
def test_float_products_leave_c(shape):
    m, n, k = shape
    for dt in (torch.float32, torch.bfloat16, torch.float16):
        scheds = [None, sm.make_schedule(tile=128, split_k=4)]
        if dt != torch.float32:
            scheds.append(sm.make_schedule(tile=256, split_k=2))
        else:
            scheds += [sm.make_schedule(precision=sm.PREC_FP16X3), sm.make_schedule(tile=128, split_k=2,
                                                                                     precision=sm.PREC_BF16X3)]
        for s in scheds:
            A = torch.empty((m, k), dtype=dt, device="cuda")
            B = torch.empty((k, n), dtype=dt, device="cuda")
            C0 = _c0(m, n, torch.float32)
            C = C0.clone()
            sm.semiring_mm(A, B, C, sm.PLUS_TIMES, schedule=s)
            torch.cuda.synchronize()
            assert torch.equal(C, C0), (shape, dt)
            if s is None or dt == torch.float32:
                C = C0.clone()
                sm.semiring_mm_static(A, B, C, sm.PLUS_TIMES, schedule=s)
                torch.cuda.synchronize()
                assert torch.equal(C, C0), (shape, dt, "static")


@pytest.mark.parametrize("shape", SHAPES)
def test_integer_semirings_leave_c(shape):
    m, n, k = shape
    for sr in (sm.MIN_PLUS, sm.MAX_PLUS, sm.MAX_MIN, sm.OR_AND):
        for s in (None, sm.make_schedule(tile=128, split_k=8), sm.make_schedule(tile=64, split_k=4, star_depth=2),
                  sm.make_schedule(tile=128, split_k=4, flags=sm.FLAG_PERSISTENT)):
            A = torch.empty((m, k), dtype=torch.int32, device="cuda")
            B = torch.empty((k, n), dtype=torch.int32, device="cuda")
            C0 = torch.from_numpy(si.semiring_init(sr, (m, n))).cuda() if sr != sm.MIN_PLUS else _c0(m, n, torch.int32)
            C = C0.clone()
            sm.semiring_mm(A, B, C, sr, schedule=s)
            torch.cuda.synchronize()
            assert torch.equal(C, C0), (shape, sr)


@pytest.mark.parametrize("shape", SHAPES)
def test_strassen_leaves_c(shape):
    m, n, k = shape
    for depth in (1, 2):
        for prec in (sm.PREC_BF16X3, sm.PREC_FP16X3, sm.PREC_BF16X3_HIACC):
            A = torch.empty((m, k), device="cuda")
            B = torch.empty((k, n), device="cuda")
            C0 = _c0(m, n, torch.float32)
            C = C0.clone()
            assert sm.strassen_workspace_bytes(m, n, k, depth, sm.CLASSIC, prec) == 0
            sm.strassen_mm(A, B, C, depth, sm.CLASSIC, prec)
            torch.cuda.synchronize()
            assert torch.equal(C, C0), (shape, depth, prec)


def test_batch_with_empty_problems():
    shapes = [(70, 90, 0), (0, 90, 40), (70, 0, 40), (96, 130, 70), (1, 1, 1), (300, 257, 33)]
    host, dev = [], []
    for i, (m, n, k) in enumerate(shapes):
        A = si.small_int_f32(40 + 2 * i, (m, k), 4)
        B = si.small_int_f32(41 + 2 * i, (k, n), 4)
        C0 = si.small_int_f32(90 + i, (m, n), 4)
        host.append((A, B, C0))
        dev.append((torch.from_numpy(A).cuda().to(torch.bfloat16), torch.from_numpy(B).cuda().to(torch.bfloat16),
                    torch.from_numpy(C0).cuda()))
    ws = torch.empty(max(sm.batched_workspace_bytes(dev), 1), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, workspace=ws)
    torch.cuda.synchronize()
    for (A, B, C0), (_, _, C) in zip(host, dev):
        ref = C0.astype(np.int64) + oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
        assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), A.shape
