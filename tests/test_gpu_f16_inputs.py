"""GPU parity of the fp16-input (+,x) product (MM_DT_F16: A, B binary16, C
float, fp16 MFMA with fp32 accumulation) through mm_semiring and the
persistent batched launch, against the oracle.

Exactness pins: integers of up to 11 significant bits are exact in fp16
(but not in bf16, which keeps 8), so a product of such an A with a B of
entries in {-1, 0, 1} whose partial sums stay below 2^24 must come back
bit for bit; that fails if any stage rounds through bf16.  Random N(0,1)
operands rounded to fp16 are checked against the float64 product of the
exact fp16 values within the fp32 accumulation bound.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402


def wide_int_case(seed, m, n, k):
    g = np.random.default_rng(seed)
    A = g.integers(-2047, 2048, (m, k)).astype(np.float32)  # 11 significant bits
    B = g.integers(-1, 2, (k, n)).astype(np.float32)
    C0 = g.integers(-8, 9, (m, n)).astype(np.float32)
    assert 2047 * k + 8 < 2 ** 24
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    return A, B, C0, ref


def f16(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda().to(torch.float16)


@pytest.mark.parametrize("shape", [(1, 1, 1), (33, 17, 65), (257, 129, 300), (300, 270, 1031)])
def test_f16_semiring_eleven_bit_integers_bit_exact(shape):
    m, n, k = shape
    A, B, C0, ref = wide_int_case(m + n + k, m, n, k)
    for tile in (32, 64, 128, 256):
        for split in (1, 2, 4):
            s = sm.make_schedule(tile=tile, split_k=split)
            wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F16, m, n, k, s)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda") if wsb else None
            dC = torch.from_numpy(C0).cuda()
            sm.semiring_mm(f16(A), f16(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
            torch.cuda.synchronize()
            assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (tile, split)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("shape", [(257, 129, 300), (1000, 777, 1031), (64, 300, 17), (512, 512, 4096)])
def test_one_plane_tiles_match_staged_tiles(dtype, shape):
    # 16-bit inputs copied once into k-tiled planes and multiplied by the
    # direct-to-LDS tiles (128 and 256 wide) give the bits of the tiles
    # staged straight from the operands (same MFMA order); k-split 1, 2, 4.
    m, n, k = shape
    tA = torch.from_numpy(si.normal_f32(m + 3, (m, k))).cuda().to(dtype)
    tB = torch.from_numpy(si.normal_f32(n + 5, (k, n))).cuda().to(dtype)
    C0 = si.normal_f32(k + 7, (m, n))
    ref = oracle.fp64_ref(tA.float().cpu().numpy(), tB.float().cpu().numpy(), C0)
    for tile in (128, 256):
        for split in (1, 2, 4):
            outs = []
            for flags in (0, sm.FLAG_SPLIT_IN_KERNEL):
                s = sm.make_schedule(tile=tile, split_k=split, flags=flags)
                wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F16 if dtype == torch.float16 else sm.DT_BF16,
                                         m, n, k, s)
                assert (wsb > 0) == (flags == 0 or split > 1)
                ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
                dC = torch.from_numpy(C0).cuda()
                sm.semiring_mm(tA, tB, dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
                torch.cuda.synchronize()
                outs.append(dC.cpu().numpy())
            assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32)), (tile, split)
            assert oracle.rel_fro(outs[0], ref) < 2.0 ** -24 * np.sqrt(k) * 4, (tile, split)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16])
def test_one_plane_copies_same_bits_for_any_operand_alignment(dtype):
    # The copies into the planes read 16-byte runs (through aligned 16-byte
    # loads and shifts where a run is not aligned) where a row's run lies
    # inside the operand (A) or a whole 64 x 64 block does (B, through LDS),
    # and single values elsewhere: operands as views at odd offsets or with
    # odd row lengths give the same bits as contiguous ones.
    m, n, k = 300, 520, 1024
    tA = torch.from_numpy(si.normal_f32(31, (m, k))).cuda().to(dtype)
    tB = torch.from_numpy(si.normal_f32(32, (k, n))).cuda().to(dtype)
    C0 = si.normal_f32(33, (m, n))
    s = sm.make_schedule(tile=256, split_k=1)
    wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F16 if dtype == torch.float16 else sm.DT_BF16, m, n, k, s)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")

    def run(A, B):
        dC = torch.from_numpy(C0).cuda()
        sm.semiring_mm(A, B, dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
        torch.cuda.synchronize()
        return dC.cpu().numpy()

    ref = run(tA, tB)
    assert oracle.rel_fro(ref, oracle.fp64_ref(tA.float().cpu().numpy(), tB.float().cpu().numpy(), C0)) < \
        2.0 ** -24 * np.sqrt(k) * 4
    for pad, off in ((1, 0), (8, 1), (9, 8)):
        Aw = torch.zeros((m, k + pad), dtype=dtype, device="cuda")
        Aw[:, off:off + k] = tA
        Bw = torch.zeros((k, n + pad), dtype=dtype, device="cuda")
        Bw[:, off:off + n] = tB
        got = run(Aw[:, off:off + k], Bw[:, off:off + n])
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (pad, off)


@pytest.mark.parametrize("shape", [(8192, 8192, 64), (4096, 4096, 96), (6144, 8192, 40)])
def test_wide_single_products_in_row_bands_exact(shape):
    # Single products on 256 tiles that are 16 or 32 tiles wide run in bands
    # of tile rows, XCD x on one block of each band: the one-plane bf16 tile,
    # the register-staged bf16 tile and the BF16x3 split tile (depth 0)
    # against the oracle, small integers.
    m, n, k = shape
    A = si.small_int_f32(m + 1, (m, k))
    B = si.small_int_f32(n + 2, (k, n))
    C0 = si.small_int_f32(k + 3, (m, n))
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    s = sm.make_schedule(tile=256, split_k=1)
    wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_BF16, m, n, k, s)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    dC = torch.from_numpy(C0).cuda()
    sm.semiring_mm(torch.from_numpy(A).cuda().to(torch.bfloat16), torch.from_numpy(B).cuda().to(torch.bfloat16), dC,
                   sm.PLUS_TIMES, workspace=ws, schedule=s)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), "one plane"
    # the register-staged tile straight from the bf16 operands (no planes)
    dC = torch.from_numpy(C0).cuda()
    sm.semiring_mm(torch.from_numpy(A).cuda().to(torch.bfloat16), torch.from_numpy(B).cuda().to(torch.bfloat16), dC,
                   sm.PLUS_TIMES, schedule=sm.make_schedule(tile=256, split_k=1, flags=sm.FLAG_SPLIT_IN_KERNEL))
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), "staged"
    wsb = sm.strassen_workspace_bytes(m, n, k, 0, sm.CLASSIC, sm.PREC_BF16X3)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    dC = torch.from_numpy(C0).cuda()
    sm.strassen_mm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), dC, 0, sm.CLASSIC, sm.PREC_BF16X3,
                   workspace=ws)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), "split"


def test_bf16_planes_small_integers_bit_exact():
    # integers of magnitude <= 8 are exact in bf16; through the planes at
    # every wide tile and split, ragged and tiny shapes included
    for (m, n, k) in [(1, 1, 1), (33, 17, 65), (257, 129, 300), (300, 270, 1031)]:
        A = si.small_int_f32(m + 11, (m, k))
        B = si.small_int_f32(n + 13, (k, n))
        C0 = si.small_int_f32(k + 17, (m, n))
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        for tile in (128, 256):
            for split in (1, 2, 4):
                s = sm.make_schedule(tile=tile, split_k=split)
                wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_BF16, m, n, k, s)
                ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
                dC = torch.from_numpy(C0).cuda()
                sm.semiring_mm(torch.from_numpy(A).cuda().to(torch.bfloat16),
                               torch.from_numpy(B).cuda().to(torch.bfloat16), dC, sm.PLUS_TIMES, workspace=ws,
                               schedule=s)
                torch.cuda.synchronize()
                assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (m, n, k, tile, split)


def test_f16_semiring_normal_tolerance_and_determinism():
    m, n, k = 1000, 1031, 1024
    tA = f16(si.normal_f32(si.BASE_SEED, (m, k)))
    tB = f16(si.normal_f32(si.BASE_SEED + 1, (k, n)))
    A = tA.float().cpu().numpy()  # the oracle sees exactly the device values
    B = tB.float().cpu().numpy()
    ref = oracle.fp64_ref(A, B)
    outs = []
    for _ in range(2):
        dC = torch.zeros((m, n), dtype=torch.float32, device="cuda")
        sm.semiring_mm(tA, tB, dC, sm.PLUS_TIMES)
        torch.cuda.synchronize()
        outs.append(dC.cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    # fp32 accumulation only: 2^-24 sqrt(k) in the typical case
    assert oracle.rel_fro(outs[0], ref) < 2.0 ** -24 * np.sqrt(k) * 2


def test_f16_batched_eleven_bit_integers_bit_exact():
    # packed (128 and 256 tiles) and unpacked problems, split-K included
    g = np.random.default_rng(5)
    shapes = [tuple(int(x) for x in g.integers(1, 300, 3)) for _ in range(24)]
    shapes += [(512, 300, 1500), (260, 600, 2048), (1, 1, 1), (129, 257, 64)]
    scheds, host, dev = [], [], []
    for i, (m, n, k) in enumerate(shapes):
        A, B, C0, ref = wide_int_case(1000 + i, m, n, k)
        host.append(ref)
        dev.append((f16(A), f16(B), torch.from_numpy(C0).cuda()))
        flags = sm.FLAG_SPLIT_IN_KERNEL if i % 5 == 3 else 0
        scheds.append(sm.make_schedule(split_k=(1, 2, 4)[i % 3], flags=flags))
    ws = torch.empty(sm.batched_workspace_bytes(dev, scheds), dtype=torch.uint8, device="cuda")
    sm.batched_mm(dev, scheds, workspace=ws)
    torch.cuda.synchronize()
    for ref, (_, _, C), shape in zip(host, dev, shapes):
        assert np.array_equal(C.cpu().numpy().astype(np.int64), ref), shape


def test_f16_batched_graph_normal_tolerance():
    g = np.random.default_rng(6)
    shapes = [tuple(int(x) for x in g.integers(16, 900, 3)) for _ in range(30)] + [(700, 800, 1500)]
    trip, host = [], []
    for i, (m, n, k) in enumerate(shapes):
        tA = f16(si.normal_f32(2000 + 2 * i, (m, k)))
        tB = f16(si.normal_f32(2001 + 2 * i, (k, n)))
        host.append((tA.float().cpu().numpy(), tB.float().cpu().numpy()))
        trip.append((tA, tB, torch.zeros((m, n), dtype=torch.float32, device="cuda")))
    ws = torch.empty(sm.batched_workspace_bytes(trip), dtype=torch.uint8, device="cuda")
    graph = sm.BatchedGraph(trip, workspace=ws)
    try:
        for rep in range(3):
            for _, _, C in trip:
                C.zero_()
            graph.launch()
            torch.cuda.synchronize()
            for (A, B), (_, _, C) in zip(host, trip):
                k = A.shape[1]
                err = oracle.rel_fro(C.cpu().numpy(), oracle.fp64_ref(A, B))
                assert err < 2.0 ** -24 * np.sqrt(k) * 2 + 1e-7, (rep, A.shape, err)
    finally:
        graph.close()
