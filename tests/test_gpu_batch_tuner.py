"""The batch-aware autotuner's per-problem schedules on the GPU: every
problem of a batch run with them is bit-exact against the oracle on
small-integer inputs, and the tuned batch is no slower than the library's own
rule (the tuner only keeps a class's alternative when the whole batch gets
faster)."""
import math

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402
from paper_1911_05328_amd.tune import batch_tuner  # noqa: E402


def test_tuned_batch_bit_exact_and_not_slower():
    g = np.random.default_rng(7)
    shapes = [tuple(int(round(math.exp(g.uniform(math.log(64), math.log(1024))))) for _ in range(3))
              for _ in range(64)]
    host, dev = [], []
    for i, (m, n, k) in enumerate(shapes):
        A = si.small_int_f32(300 + 2 * i, (m, k), 4)
        B = si.small_int_f32(301 + 2 * i, (k, n), 4)
        tA = torch.from_numpy(A).cuda().to(torch.bfloat16)
        tB = torch.from_numpy(B).cuda().to(torch.bfloat16)
        host.append((A, B))
        dev.append((tA, tB, torch.zeros((m, n), device="cuda")))
    scheds, rep = batch_tuner.tune(dev)
    print("batch tuner:", {k: v for k, v in rep.items() if k != "trace"}, flush=True)
    assert len(scheds) == len(shapes)
    # re-timed in alternation with the rule: no slower beyond timing noise
    assert rep["tuned_ms"] <= rep["rule_ms"] * 1.05, rep
    for _, _, C in dev:
        C.zero_()
    ws = torch.empty(max(sm.batched_workspace_bytes(dev, scheds), 1), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, schedules=scheds, workspace=ws)
    torch.cuda.synchronize()
    for (A, B), (_, _, C) in zip(host, dev):
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
        assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), A.shape
