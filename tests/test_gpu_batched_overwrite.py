"""GPU: MM_FLAG_OVERWRITE_C in a batch -- C = A B with plain stores (the
initial C is never read), mixed in one launch with problems that accumulate,
with k-splits, with k = 0 (C becomes 0), as a direct launch and as a graph
launched twice (overwritten problems stay A B, the others reach C0 + 2 A B).
Small-integer inputs keep every case bit-exact against the oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}


@pytest.mark.parametrize("kind", ["bf16", "f32", "f16"])
@pytest.mark.parametrize("graph", [False, True])
def test_overwrite_mixed_batch_bit_exact(kind, graph):
    g = np.random.default_rng(99 + graph)
    shapes = [tuple(int(x) for x in g.integers(1, 600, 3)) for _ in range(20)]
    shapes += [(300, 280, 0), (513, 257, 1030), (64, 700, 40), (1, 1, 1)]
    host, dev, scheds = [], [], []
    for i, (m, n, k) in enumerate(shapes):
        A = g.integers(-4, 5, (m, k)).astype(np.float32)
        B = g.integers(-4, 5, (k, n)).astype(np.float32)
        C0 = g.integers(-1000, 1000, (m, n)).astype(np.float32)  # garbage for overwritten problems
        over = i % 2 == 0 or k == 0
        host.append((A, B, C0, over))
        dev.append((torch.from_numpy(A).cuda().to(TORCH_DT[kind]), torch.from_numpy(B).cuda().to(TORCH_DT[kind]),
                    torch.from_numpy(C0).cuda()))
        flags = sm.FLAG_OVERWRITE_C if over else 0
        if i % 7 == 3:
            flags |= sm.FLAG_SPLIT_IN_KERNEL
        scheds.append(sm.make_schedule(split_k=(1, 2, 4)[i % 3], flags=flags))
    ws = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    if graph:
        gr = sm.BatchedGraph(dev, schedules=scheds, workspace=ws)
        try:
            gr.launch()
            gr.launch()
        finally:
            torch.cuda.synchronize()
            gr.close()
    else:
        sm.batched_mm(dev, scheds, workspace=ws)
    torch.cuda.synchronize()
    for (A, B, C0, over), (_, _, C), shape in zip(host, dev, shapes):
        Ai, Bi = A.astype(np.int64), B.astype(np.int64)
        prod = oracle.brute(sm.PLUS_TIMES, Ai, Bi)
        if over:
            want = prod
        else:
            want = C0.astype(np.int64) + prod * (2 if graph else 1)
        assert np.array_equal(C.cpu().numpy().astype(np.int64), want), (kind, graph, shape, over)


def test_overwrite_flag_is_batched_only():
    s = sm.make_schedule(flags=sm.FLAG_OVERWRITE_C)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, 64, 64, 64, 1 << 20, s)[0] == sm.MM_ERR_INVALID_ARG
