"""Seeded random sweep of mm_batched: batches of uneven problems of one
dtype (fp32 through BF16x3, bf16, fp16) with random per-problem schedules
(k-split, tile 128 / 256, opting out of packing), on small-integer inputs
whose products and partial sums are exact in every format, so each problem
is bit-exact against the oracle; every other batch also runs as a captured
graph, launched twice (the second launch adds the product once more)."""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


def test_random_batches_bit_exact():
    g = np.random.default_rng(4242)
    for b in range(int(os.environ.get("STARMM_BATCH_SWEEP", "24"))):
        kind = ("f32", "bf16", "f16")[b % 3]
        count = int(g.integers(1, 41))
        host, dev, scheds = [], [], []
        for _ in range(count):
            m, n, k = (int(x) for x in np.exp(g.uniform(0, np.log(700), 3)).round().clip(1, 700))
            A = g.integers(-4, 5, (m, k)).astype(np.float32)
            B = g.integers(-4, 5, (k, n)).astype(np.float32)
            C0 = g.integers(-8, 9, (m, n)).astype(np.float32)
            host.append((A, B, C0))
            dev.append((torch.from_numpy(A).cuda().to(TORCH_DT[kind]), torch.from_numpy(B).cuda().to(TORCH_DT[kind]),
                        torch.from_numpy(C0).cuda()))
            flags = sm.FLAG_SPLIT_IN_KERNEL if g.random() < 0.2 else 0
            tile = int(g.choice([0, 128, 256])) if not flags else int(g.choice([0, 128]))
            scheds.append(sm.make_schedule(tile=tile, split_k=int(g.choice([0, 1, 2, 4, 8])), flags=flags))
        use = scheds if g.random() < 0.7 else None
        ws = torch.empty(max(sm.batched_workspace_bytes(dev, use), 1), dtype=torch.uint8, device="cuda")
        graph = b % 2 == 1
        if graph:
            gr = sm.BatchedGraph(dev, schedules=use, workspace=ws)
            try:
                gr.launch()
                gr.launch()
            finally:
                torch.cuda.synchronize()
                gr.close()
        else:
            sm.batched_mm(dev, use, workspace=ws)
        torch.cuda.synchronize()
        for i, ((A, B, C0), (_, _, C)) in enumerate(zip(host, dev)):
            Ai, Bi = A.astype(np.int64), B.astype(np.int64)
            want = oracle.brute(sm.PLUS_TIMES, Ai, Bi, C0.astype(np.int64))
            if graph:
                want = oracle.brute(sm.PLUS_TIMES, Ai, Bi, want)
            assert np.array_equal(C.cpu().numpy().astype(np.int64), want), (b, kind, i, A.shape, B.shape,
                                                                             use[i].as_dict() if use else None)
