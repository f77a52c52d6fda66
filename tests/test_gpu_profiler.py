"""GPU: the library's own launch profiler (mm_profile_*) and the
microbenchmarks behind measured_peaks (mm_microbench).

The profiler records HIP events on the launch stream around each kernel
family; its totals must cover the families a call launches, count each
launch once, and add up to no more than the wall time around them.  The
microbenchmarks must land between sane fractions of the datasheet figures
(HBM 8 TB/s, bf16 MFMA 2.5 PFLOP/s, fp32 MFMA 157.3 TFLOP/s, int32 VALU
78.6 T lane-instructions/s: 256 CUs x 128 lanes x 2.4 GHz)."""
import time

import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402


def test_profiler_counts_and_times_launches():
    n = 2048
    A = torch.from_numpy(si.normal_f32(1, (n, n))).cuda()
    B = torch.from_numpy(si.normal_f32(2, (n, n))).cuda()
    C = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    ws = torch.empty(sm.strassen_workspace_bytes(n, n, n, 1, sm.CLASSIC, sm.PREC_BF16X3), dtype=torch.uint8,
                     device="cuda")
    sm.strassen_mm(A, B, C, 1, sm.CLASSIC, sm.PREC_BF16X3, workspace=ws)  # warm
    torch.cuda.synchronize()
    sm.profile_enable(True)
    try:
        sm.profile_reset()
        t0 = time.perf_counter()
        for _ in range(5):
            sm.strassen_mm(A, B, C, 1, sm.CLASSIC, sm.PREC_BF16X3, workspace=ws)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        prof = sm.profile_summary()
    finally:
        sm.profile_enable(False)
    assert prof["bf16x3_tile"][0] == 5 and prof["strassen_post"][0] == 5
    assert prof["strassen_pre"][0] == 10  # one pre-addition pass per operand
    total = sum(ms for _, ms in prof.values())
    assert all(ms > 0 for _, ms in prof.values())
    assert total <= wall_ms * 1.05
    sm.profile_reset()
    assert sm.profile_summary() == {}


def test_measured_peaks_are_plausible():
    peaks = sm.measured_peaks()
    assert 1.0e12 < peaks["copy_bytes"] < 8.0e12
    assert 0.5e15 < peaks["mfma_bf16_flops"] < 2.5e15 * 1.02
    assert 30e12 < peaks["mfma_f32_flops"] < 157.3e12 * 1.02
    assert 10e12 < peaks["valu_i32_ops"] < 256 * 128 * 2.4e9 * 1.02
