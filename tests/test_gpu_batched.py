"""GPU parity of the persistent batched launch (mm_batched and its hipGraph).

Every problem of a batch is checked against the oracle: bit-exact on
small-integer inputs (exact in bf16, partial sums below 2^24), within a
relative Frobenius tolerance on the full 512-problem log-uniform batch.
Graph replays are interleaved with eager work and synchronisations and
every replay is compared with the eager result.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402


def make_batch(shapes, seed, dtype, bound=None):
    host, dev = [], []
    for i, (m, n, k) in enumerate(shapes):
        if bound is None:
            A = si.normal_f32(seed + 3 * i, (m, k))
            B = si.normal_f32(seed + 3 * i + 1, (k, n))
        else:
            A = si.small_int_f32(seed + 3 * i, (m, k), bound)
            B = si.small_int_f32(seed + 3 * i + 1, (k, n), bound)
        C0 = np.zeros((m, n), np.float32)
        tA = torch.from_numpy(A).cuda().to(dtype)
        tB = torch.from_numpy(B).cuda().to(dtype)
        tC = torch.from_numpy(C0).cuda()
        # the oracle sees exactly the values the GPU gets
        host.append((tA.float().cpu().numpy(), tB.float().cpu().numpy()))
        dev.append((tA, tB, tC))
    return host, dev


def ragged_shapes(count, seed, hi=300):
    g = np.random.default_rng(seed)
    return [tuple(int(x) for x in g.integers(1, hi, 3)) for _ in range(count)]


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
def test_batched_small_integers_bit_exact(dtype):
    shapes = ragged_shapes(40, 1) + [(1, 1, 1), (128, 128, 128), (129, 257, 64), (7, 400, 3)]
    host, dev = make_batch(shapes, 100, dtype, bound=8)
    ws = torch.empty(max(sm.batched_workspace_bytes(dev), 1), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, workspace=ws)
    torch.cuda.synchronize()
    for (A, B), (_, _, C) in zip(host, dev):
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
        assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), A.shape


def test_batched_split_k_deterministic_and_exact():
    shapes = [(100, 90, 3000), (256, 256, 2048), (33, 17, 5000), (300, 129, 64)] + ragged_shapes(12, 2)
    host, dev = make_batch(shapes, 200, torch.bfloat16, bound=4)
    scheds = [sm.make_schedule(split_k=s) for s in ([8, 4, 16, 2] + [1, 2, 4] * 4)]
    ws = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    results = []
    for _ in range(2):
        for _, _, C in dev:
            C.zero_()
        sm.batched_mm(dev, scheds, workspace=ws)
        torch.cuda.synchronize()
        results.append([C.cpu().numpy().copy() for _, _, C in dev])
    for (A, B), r0, r1 in zip(host, results[0], results[1]):
        assert np.array_equal(r0.view(np.uint32), r1.view(np.uint32))
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
        assert np.array_equal(r0.astype(np.int64), ref)


def test_batched_graph_replays_match_eager():
    shapes = ragged_shapes(60, 3, hi=700)
    host, dev = make_batch(shapes, 300, torch.bfloat16)
    scheds = [sm.make_schedule(split_k=(4 if k > 400 else 1)) for (_, _, k) in shapes]
    ws_e = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, scheds, workspace=ws_e)
    torch.cuda.synchronize()
    eager = [C.cpu().numpy().copy() for _, _, C in dev]
    ws_g = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    g = sm.BatchedGraph(dev, scheds, workspace=ws_g)
    try:
        for rep in range(4):
            for _, _, C in dev:
                C.zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            x = torch.randn(256, 256, device="cuda")  # unrelated eager work between replays
            (x @ x).sum().item()
            for e, (_, _, C) in zip(eager, dev):
                assert np.array_equal(C.cpu().numpy().view(np.uint32), e.view(np.uint32)), rep
    finally:
        g.close()
    for (A, B), e in zip(host, eager):
        ref = oracle.fp64_ref(A, B)
        assert oracle.rel_fro(e, ref) < 2.0 ** -24 * np.sqrt(A.shape[1]) + 1e-7


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_batched_in_launch_pack_replays_exact_and_no_wait_gave_up(dtype):
    # bf16 / fp16 batches pack their operands in the first phase of the
    # persistent launch (a tile waits for its problem's planes): graph
    # replays on changing inputs stay exact, mixing packed 256 / 128 tiles
    # (the 128 kind runs after the packing launch), staged problems and
    # k-splits, and the control words of the packing kind (workspace offset
    # 0: 3 kinds x 8 queues of {next, done, pack_next, error} uint32) show
    # every counter reset and no bounded wait given up.
    shapes = ragged_shapes(40, 21, hi=600) + [(700, 650, 900), (1, 1, 1), (300, 257, 64)]
    host, dev = make_batch(shapes, 1300, dtype, bound=4)
    scheds = [sm.make_schedule(tile=(0, 0, 128)[i % 3], split_k=(1, 2, 1, 4)[i % 4],
                               flags=(sm.FLAG_SPLIT_IN_KERNEL if i % 7 == 3 else 0))
              for i in range(len(shapes))]
    for i, s in enumerate(scheds):
        if s.flags and s.tile == 128:
            s.tile = 0  # staged problems run on their own kind
    ws = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    g = sm.BatchedGraph(dev, scheds, workspace=ws)
    try:
        for rep in range(3):
            scale = rep + 1  # exact: |entries| <= 12, partial sums < 2^24
            for (A, B), (tA, tB, tC) in zip(host, dev):
                tA.copy_(torch.from_numpy(A * scale).cuda().to(dtype))
                tC.zero_()
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for (A, B), (_, _, C) in zip(host, dev):
                ref = oracle.brute(oracle.PLUS_TIMES, (A * scale).astype(np.int64), B.astype(np.int64))
                assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), (rep, A.shape)
            ctl = ws[: 3 * 8 * 16].cpu().numpy().view(np.uint32).reshape(3, 8, 4)
            assert not ctl.any(), ctl  # next / done / pack_next reset, error 0
    finally:
        g.close()


def test_batched_rejects_bad_arguments():
    A = torch.zeros((8, 8), dtype=torch.bfloat16, device="cuda")
    C = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(sm.StarmmError):
        sm.batched_mm([(A, A, C)], workspace=None)  # no workspace for the tables
    with pytest.raises(sm.StarmmError):
        ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
        sm.batched_mm([(A, A, C)], [sm.make_schedule(strassen_depth=1)], workspace=ws)


def test_batched_512_log_uniform_sampled():
    # The uneven batch: 512 problems, m, n, k each log-uniform in [64, 4096],
    # bf16 N(0,1) inputs, fp32 accumulation, one graph replay; against the
    # float64 oracle of the bf16 values on whole rows: one in every 256-row
    # tile row of every problem (at an offset inside the tile that varies
    # with the problem and the tile row) plus the last, so every output tile
    # of every problem has a checked row.
    shapes = [tuple(int(v) for v in r) for r in si.batched_shapes(si.BASE_SEED, 512)]
    dev, host_rows = [], []
    for i, (m, n, k) in enumerate(shapes):
        tA = torch.randn(m, k, device="cuda", generator=torch.Generator(device="cuda").manual_seed(i)).to(torch.bfloat16)
        tB = torch.randn(k, n, device="cuda", generator=torch.Generator(device="cuda").manual_seed(10_000 + i)).to(torch.bfloat16)
        tC = torch.zeros((m, n), dtype=torch.float32, device="cuda")
        rows = np.unique([min(m - 1, t * 256 + (37 * i + 53 * t) % 256) for t in range(-(-m // 256))] + [m - 1])
        dev.append((tA, tB, tC))
        host_rows.append(rows)
    ws = torch.empty(sm.batched_workspace_bytes(dev), dtype=torch.uint8, device="cuda")
    gr = sm.BatchedGraph(dev, workspace=ws)
    try:
        gr.launch()
        torch.cuda.synchronize()
    finally:
        gr.close()
    for (tA, tB, tC), rows in zip(dev, host_rows):
        A = tA[torch.from_numpy(rows).cuda()].float().cpu().numpy()
        B = tB.float().cpu().numpy()
        ref = oracle.fp64_rows(A, B, np.arange(len(rows)))
        got = tC[torch.from_numpy(rows).cuda()].cpu().numpy()
        assert oracle.rel_fro(got, ref) < 2.0 ** -24 * np.sqrt(tA.shape[1]) * 2 + 1e-7


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
def test_batched_packed_and_unpacked_problems_agree_exactly(dtype):
    # Packed problems (operands rewritten as k-tiled planes) and problems
    # staged straight from their operands (MM_FLAG_SPLIT_IN_KERNEL) in one
    # launch; ragged, unaligned shapes with k-splits; both exact.
    shapes = ragged_shapes(30, 9, hi=520) + [(1, 1, 1), (256, 130, 33), (31, 300, 1000), (64, 64, 8)]
    host, dev = make_batch(shapes, 900, dtype, bound=4)
    scheds = [sm.make_schedule(split_k=(1, 2, 4)[i % 3], flags=(sm.FLAG_SPLIT_IN_KERNEL if i % 2 else 0))
              for i in range(len(shapes))]
    ws = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, scheds, workspace=ws)
    torch.cuda.synchronize()
    for (A, B), (_, _, C) in zip(host, dev):
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
        assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), A.shape


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float32])
def test_batched_wide_tiles_exact(dtype):
    # 256-wide tiles over packed planes (chosen explicitly here; the default
    # picks them for large problems): ragged edges, k-splits, both dtypes.
    shapes = [(256, 256, 64), (300, 513, 100), (257, 300, 1000), (512, 512, 33), (700, 260, 17)]
    host, dev = make_batch(shapes, 1200, dtype, bound=4)
    scheds = [sm.make_schedule(tile=256, split_k=s) for s in (1, 2, 4, 1, 2)]
    ws = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, scheds, workspace=ws)
    torch.cuda.synchronize()
    for (A, B), (_, _, C) in zip(host, dev):
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
        assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), A.shape
