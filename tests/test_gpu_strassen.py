"""GPU parity of the split-precision (BF16x3) base product and of the
Strassen / Strassen-Winograd levels against the oracle.

Exactness pins: with integer inputs chosen so that every Strassen operand
is an integer of magnitude <= 256 (exact in bf16, so the lo part is zero)
and every partial sum stays below 2^24 (exact in fp32), any correct
implementation returns the integer product bit for bit.  Random inputs are
checked against the float64 oracle within a relative Frobenius tolerance
derived from the split (each product carries ~2^-16 relative error) and
the growth of Strassen's error per level (about 2x classic, 2.6x Winograd).
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

MiB = 1 << 20


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_strassen(A, B, C0, depth, variant, prec):
    m, k = A.shape
    n = B.shape[1]
    wsb = sm.strassen_workspace_bytes(m, n, k, depth, variant, prec)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda") if wsb else None
    dC = dev(C0)
    sm.strassen_mm(dev(A), dev(B), dC, depth, variant, prec, workspace=ws)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def exact_bound(variant, depth, k):
    """Largest integer bound b (inputs in [-b, b]) that keeps every operand
    <= 256 in magnitude and every partial sum below 2^24."""
    growth = (2 if variant == sm.CLASSIC else 4) ** depth  # terms per leaf operand
    outputs = 4 ** depth  # products summed into one output block (upper bound)
    leaf_k = -(-k // 2 ** depth)
    b = 8
    while b > 1 and (b * growth > 256 or leaf_k * (b * growth) ** 2 * outputs >= 2 ** 24):
        b //= 2
    return b


PRECS = [sm.PREC_F32, sm.PREC_BF16X3, sm.PREC_BF16X3_HIACC]


@pytest.mark.parametrize("shape", [(1, 1, 1), (33, 17, 65), (128, 128, 128), (257, 129, 300), (640, 384, 1024)])
def test_bf16x3_depth0_small_integers_bit_exact(shape):
    m, n, k = shape
    A = si.small_int_f32(1, (m, k))
    B = si.small_int_f32(2, (k, n))
    C0 = si.small_int_f32(3, (m, n))
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    for tile in (32, 64, 128, 256):
        for s in (1, 2):
            dC = dev(C0)
            ws = torch.empty(32 * MiB, dtype=torch.uint8, device="cuda")
            sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws,
                           schedule=sm.make_schedule(tile=tile, split_k=s, precision=sm.PREC_BF16X3))
            torch.cuda.synchronize()
            assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (tile, s)


def test_bf16_inputs_bit_exact():
    m, n, k = 200, 136, 264
    A = si.small_int_f32(4, (m, k))
    B = si.small_int_f32(5, (k, n))
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64))
    for tile in (32, 64, 128, 256):
        dC = torch.zeros((m, n), dtype=torch.float32, device="cuda")
        sm.semiring_mm(dev(A).to(torch.bfloat16), dev(B).to(torch.bfloat16), dC, sm.PLUS_TIMES,
                       schedule=sm.make_schedule(tile=tile))
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), tile


def test_bf16x3_split_error_matches_emulation():
    # The device split (hardware RNE) must give the same hi/lo as the
    # oracle's bit-level RNE: compare C from the kernel against the float64
    # value of Ah Bh + Ah Bl + Al Bh; only fp32 accumulation rounding remains.
    m, n, k = 96, 80, 512
    A = si.normal_f32(6, (m, k))
    B = si.normal_f32(7, (k, n))
    dC = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES,
                   schedule=sm.make_schedule(tile=32, split_k=1, precision=sm.PREC_BF16X3))
    torch.cuda.synchronize()
    emu = oracle.split3_product_f64(A, B)
    exact = oracle.fp64_ref(A, B)
    got = dC.cpu().numpy()
    # distance to the emulated split product: fp32 accumulation only (~1e-7)
    assert oracle.rel_fro(got, emu) < 5e-7
    # the split itself: ~2^-16 per product, averaging out below 1e-5
    assert oracle.rel_fro(got, exact) < 1e-5


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("prec", PRECS)
def test_strassen_small_integers_bit_exact(variant, depth, prec):
    for (m, n, k) in [(256, 256, 256), (257, 129, 99), (37, 300, 65), (8, 8, 8)]:
        b = exact_bound(variant, depth, k)
        g = np.random.default_rng(m + n + k + depth)
        A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
        B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
        C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        got = run_strassen(A, B, C0, depth, variant, prec)
        assert np.array_equal(got.astype(np.int64), ref), (m, n, k, b)


# Relative Frobenius tolerances for N(0,1) inputs.  Two error sources add:
# fp32 accumulation over k terms, bounded in the typical case by
# 2^-24 sqrt(k), and the BF16x3 split, which drops lo*lo and rounds lo
# (~2^-16 per product; an exact-arithmetic emulation shows 4.4e-6 at
# depth 0, and we allow twice that).  Each Strassen level multiplies the
# error by about 2 (classic) or 2.6 (Winograd); we allow 2.0 / 2.7.
def tolerance(prec, variant, depth, k=1024):
    base = 2.0 ** -24 * np.sqrt(k) + (0.0 if prec == sm.PREC_F32 else 9e-6)
    growth = 2.0 if variant == sm.CLASSIC else 2.7
    return base * growth ** depth


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("depth", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", PRECS)
def test_strassen_normal_tolerance_and_determinism(variant, depth, prec):
    m, n, k = 1000, 1031, 1024
    A = si.normal_f32(si.BASE_SEED, (m, k))
    B = si.normal_f32(si.BASE_SEED + 1, (k, n))
    C0 = np.zeros((m, n), np.float32)
    got = run_strassen(A, B, C0, depth, variant, prec)
    again = run_strassen(A, B, C0, depth, variant, prec)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    err = oracle.rel_fro(got, oracle.fp64_ref(A, B))
    assert err < tolerance(prec, variant, depth), err


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("prec", [sm.PREC_BF16X3, sm.PREC_FP16X3])
@pytest.mark.parametrize("k", [520, 518])
@pytest.mark.parametrize("depth", [0, 1])
def test_pre_addition_same_bits_for_any_operand_alignment(variant, prec, k, depth):
    # One level's A-side pre-addition reads 16-byte runs of A's rows, and its
    # post-addition updates 16-byte runs of C's rows, where a block's columns
    # and the row length allow it (k = 520: every block of A; k = 518 and
    # n = 1030: the first block column only) and single elements elsewhere
    # (operands as views at odd offsets or with odd row lengths).  At depth 0
    # the splits into planes read in-range runs through aligned 16-byte
    # loads and shifts.  Every way gives the same values, so C is the same
    # bit for bit whatever the alignment.
    m, n = 300, 1030
    A = si.normal_f32(si.BASE_SEED + 2, (m, k))
    B = si.normal_f32(si.BASE_SEED + 3, (k, n))
    C0 = np.zeros((m, n), np.float32)
    ref = run_strassen(A, B, C0, depth, variant, prec)
    assert oracle.rel_fro(ref, oracle.fp64_ref(A, B)) < tolerance(prec, variant, depth, k)
    wsb = sm.strassen_workspace_bytes(m, n, k, depth, variant, prec)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    dA, dB = dev(A), dev(B)
    for pad, off in ((1, 0), (4, 1), (5, 3)):
        Aw = torch.zeros((m, k + pad), device="cuda")
        Aw[:, off:off + k] = dA
        Bw = torch.zeros((k, n + pad), device="cuda")
        Bw[:, off:off + n] = dB
        Cw = torch.zeros((m, n + pad), device="cuda")
        sm.strassen_mm(Aw[:, off:off + k], Bw[:, off:off + n], Cw[:, off:off + n], depth, variant, prec,
                       workspace=ws)
        torch.cuda.synchronize()
        got = Cw[:, off:off + n].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (pad, off)


def test_strassen_accumulates_into_c():
    m = n = k = 200
    A = si.normal_f32(1, (m, k))
    B = si.normal_f32(2, (k, n))
    C0 = si.normal_f32(3, (m, n))
    got = run_strassen(A, B, C0, 2, sm.WINOGRAD, sm.PREC_BF16X3_HIACC)
    ref = oracle.fp64_ref(A, B, C0)
    assert oracle.rel_fro(got, ref) < tolerance(sm.PREC_BF16X3, sm.WINOGRAD, 2, k=k)
    # C0 was really added: the error relative to A B alone is large
    assert oracle.rel_fro(got, oracle.fp64_ref(A, B)) > 1e-2


_FULL_REFS = {}


def _full_size_inputs(data, n=8192):
    """The n = 8192 inputs of a data set and the oracle's float64 product of
    them (computed once per set)."""
    if data not in _FULL_REFS:
        if data == "normal":
            A = si.normal_f32(si.BASE_SEED, (n, n))
            B = si.normal_f32(si.BASE_SEED + 1, (n, n))
        else:
            A = si.row_scaled_normal_f32(si.BASE_SEED, (n, n))
            B = si.row_scaled_normal_f32(si.BASE_SEED + 1, (n, n))
        _FULL_REFS.clear()
        _FULL_REFS[data] = (A, B, oracle.fp64_ref(A, B))
    return _FULL_REFS[data]


@pytest.mark.parametrize("depth,variant", [(1, sm.CLASSIC), (1, sm.WINOGRAD), (2, sm.WINOGRAD), (3, sm.WINOGRAD)])
@pytest.mark.parametrize("data", ["normal", "rows_scaled"])
def test_strassen_full_size_full_matrix(depth, variant, data):
    # n = 8192 Strassen (classic depth 1 is the benchmarked configuration)
    # over the BF16x3 base product, against the oracle's float64 product on
    # the whole matrix.
    n = 8192
    A, B, ref = _full_size_inputs(data, n)
    C0 = np.zeros((n, n), np.float32)
    print(f"Strassen n=8192 {data} depth {depth} variant {variant}", flush=True)
    got = run_strassen(A, B, C0, depth, variant, sm.PREC_BF16X3)
    assert np.isfinite(got).all()
    err = oracle.rel_fro(got, ref)
    assert err < tolerance(sm.PREC_BF16X3, variant, depth, k=n), err
    if depth == 1 and variant == sm.CLASSIC and data == "normal":
        # the benchmark's error target on these inputs
        assert err < 1e-5, err


@pytest.mark.parametrize("depth", [1, 2])
def test_strassen_schedules_leaf_tile_and_split_exact(depth):
    # Strassen through mm_semiring schedules: the leaf products take the
    # schedule's tile and k-split (temporaries per leaf, ordered merge).
    m, n, k = 300, 260, 512
    b = exact_bound(sm.WINOGRAD, depth, k)
    g = np.random.default_rng(depth)
    A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
    B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
    C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    for tile in (32, 64, 128, 256):
        for split in (1, 2, 8):
            s = sm.make_schedule(tile=tile, split_k=split, strassen_depth=depth, variant=sm.WINOGRAD,
                                 precision=sm.PREC_BF16X3)
            wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
            dC = dev(C0)
            sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
            torch.cuda.synchronize()
            assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (tile, split)


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
def test_strassen_leaf_launch_of_256_items_per_leaf_exact(variant):
    # 2048^3 at depth 1 with 128 leaf tiles split 4 ways: 64 tiles x 4
    # slices = 256 workgroups per leaf, so each XCD takes its eighth of one
    # leaf after another; small integers keep every value exact.
    m = n = k = 2048
    b = exact_bound(variant, 1, k)
    g = np.random.default_rng(2048 + variant)
    A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
    B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
    C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    for tile, split in ((128, 4), (256, 1), (128, 1)):
        s = sm.make_schedule(tile=tile, split_k=split, strassen_depth=1, variant=variant, precision=sm.PREC_BF16X3)
        wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
        dC = dev(C0)
        sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (tile, split)


@pytest.mark.parametrize("shape", [(257, 129, 300), (1000, 520, 1031), (64, 64, 8)])
def test_bf16x3_planes_equal_in_kernel_split(shape):
    # The workspace path (operands split once into bf16 planes, B transposed)
    # and the in-kernel split compute the same hi/lo values and feed the MFMAs
    # the same operands in the same order: results are bitwise identical.
    m, n, k = shape
    A = si.normal_f32(21, (m, k))
    B = si.normal_f32(22, (k, n))
    C0 = si.normal_f32(23, (m, n))
    for tile in (32, 128, 256):
        outs = []
        for flags in (0, sm.FLAG_SPLIT_IN_KERNEL):
            s = sm.make_schedule(tile=tile, split_k=1, precision=sm.PREC_BF16X3, flags=flags)
            wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda") if wsb else None
            dC = dev(C0)
            sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
            torch.cuda.synchronize()
            outs.append(dC.cpu().numpy())
        assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32)), tile
        assert oracle.rel_fro(outs[0], oracle.fp64_ref(A, B, C0)) < tolerance(sm.PREC_BF16X3, sm.WINOGRAD, 0, k)


@pytest.mark.parametrize("split", [1, 2, 4])
def test_bf16x3_planes_wide_tile_stage_counts_exact(split):
    # The 256-wide planes tile streams k in 16-deep stages, four buffers
    # deep, with separate code for the first stages and the last ones: sweep
    # k across 1..10 stages (ragged and whole), with ragged m and n so edge
    # tiles clamp their rows, and k-slices so stages start mid-matrix.
    m, n = 300, 270
    for k in (1, 15, 16, 17, 33, 48, 49, 64, 65, 112, 113, 128, 129, 144, 160):
        A = si.small_int_f32(31, (m, k))
        B = si.small_int_f32(32, (k, n))
        C0 = si.small_int_f32(33, (m, n))
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        s = sm.make_schedule(tile=256, split_k=split, precision=sm.PREC_BF16X3)
        wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)  # includes the planes
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
        dC = dev(C0)
        sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (k, split)


def run_schedule(A, B, C0, s):
    m, k = A.shape
    n = B.shape[1]
    wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    dC = dev(C0)
    sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


@pytest.mark.parametrize("top", [1, 2, 3])
@pytest.mark.parametrize("depth", [1, 2])
@pytest.mark.parametrize("prec", [sm.PREC_F32, sm.PREC_BF16X3, sm.PREC_FP16X3])
def test_star_strassen_small_integers_bit_exact(top, depth, prec):
    # STAR-Strassen: 8-way levels above the Strassen levels, with ragged
    # sizes whose blocks differ by one row / column / k and blocks that are
    # empty (m = 5 at three 8-way levels).
    for (m, n, k) in [(300, 260, 513), (5, 77, 40), (129, 1, 257)]:
        b = exact_bound(sm.WINOGRAD, depth, k)
        g = np.random.default_rng(m + n + k + top)
        A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
        B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
        C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        s = sm.make_schedule(strassen_depth=depth, star_depth=top, variant=sm.WINOGRAD, precision=prec)
        got = run_schedule(A, B, C0, s)
        assert np.array_equal(got.astype(np.int64), ref), (m, n, k)


@pytest.mark.parametrize("top", [1, 2])
@pytest.mark.parametrize("prec", [sm.PREC_BF16X3, sm.PREC_FP16X3])
def test_star_strassen_normal_tolerance_and_determinism(top, prec):
    # Each output block sums 2^top k-slice products, each with the error of a
    # Strassen product of depth 1 over k / 2^top: the depth-1 tolerance holds.
    m, n, k = 1000, 1031, 1024
    A = si.normal_f32(si.BASE_SEED, (m, k))
    B = si.normal_f32(si.BASE_SEED + 1, (k, n))
    C0 = si.normal_f32(si.BASE_SEED + 2, (m, n))
    s = sm.make_schedule(strassen_depth=1, star_depth=top, variant=sm.WINOGRAD, precision=prec)
    got = run_schedule(A, B, C0, s)
    again = run_schedule(A, B, C0, s)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    ref = oracle.star_strassen(A.astype(np.float64), B.astype(np.float64), top, 1, oracle.STRASSEN_WINOGRAD, C0)
    assert oracle.rel_fro(ref, oracle.fp64_ref(A, B, C0)) < 1e-13
    tol = tolerance(sm.PREC_BF16X3 if prec == sm.PREC_BF16X3 else sm.PREC_F32, sm.WINOGRAD, 1, k)
    assert oracle.rel_fro(got, ref) < tol


# ---- depth-first (SAR-Strassen) levels on top of breadth-first ones

LAYOUT_PRECS = [sm.PREC_F32, sm.PREC_BF16X3, sm.PREC_BF16X3_HIACC, sm.PREC_FP16X3]


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("depth", [1, 2, 3])
@pytest.mark.parametrize("prec", LAYOUT_PRECS)
def test_strassen_depth_first_levels_small_integers_bit_exact(variant, depth, prec):
    # t of the depth levels depth-first on top (7^t rounds, each adding its
    # product into C at once): integers keep every operand exact in bf16 /
    # fp16 and every partial sum below 2^24, so each layout gives the
    # integer product bit for bit, ragged and tiny sizes included.
    for (m, n, k) in [(256, 256, 256), (257, 129, 99), (37, 300, 65), (8, 8, 8)]:
        b = exact_bound(variant, depth, k)
        g = np.random.default_rng(m + n + k + depth)
        A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
        B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
        C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        for t in range(1, depth + 1):
            print(f"layout t={t} depth {depth} variant {variant} prec {prec} shape {(m, n, k)}", flush=True)
            s = sm.make_schedule(strassen_depth=depth, variant=variant, precision=prec,
                                 strassen_layout=sm.strassen_layout((1 << t) - 1))
            got = run_schedule(A, B, C0, s)
            assert np.array_equal(got.astype(np.int64), ref), (m, n, k, t)


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_depth_first_levels_tolerance_and_determinism(variant, depth):
    # Random inputs: each layout against the oracle's recursion with the same
    # levels depth-first (its float64 result equals the classical product to
    # 1e-13), within the breadth-first tolerance; two runs give the same bits.
    m, n, k = 1000, 1031, 1024
    A = si.normal_f32(si.BASE_SEED, (m, k))
    B = si.normal_f32(si.BASE_SEED + 1, (k, n))
    C0 = si.normal_f32(si.BASE_SEED + 2, (m, n))
    exact = oracle.fp64_ref(A, B, C0)
    for t in range(1, depth + 1):
        mask = (1 << t) - 1
        ref, _ = oracle.strassen_layout(A.astype(np.float64), B.astype(np.float64), depth,
                                        oracle.STRASSEN_CLASSIC if variant == sm.CLASSIC else oracle.STRASSEN_WINOGRAD,
                                        mask, C0.astype(np.float64))
        assert oracle.rel_fro(ref, exact) < 1e-13
        for prec in (sm.PREC_BF16X3, sm.PREC_FP16X3):
            s = sm.make_schedule(strassen_depth=depth, variant=variant, precision=prec,
                                 strassen_layout=sm.strassen_layout(mask))
            got = run_schedule(A, B, C0, s)
            again = run_schedule(A, B, C0, s)
            assert np.array_equal(got.view(np.uint32), again.view(np.uint32)), (t, prec)
            assert oracle.rel_fro(got, ref) < tolerance(sm.PREC_BF16X3, variant, depth, k), (t, prec)


def test_mm_strassen_small_workspace_takes_depth_first_levels():
    # mm_strassen with less workspace than the breadth-first layout: the
    # planner's layout (the fewest depth-first levels on top that fit) gives
    # the same bits as the schedule naming that layout, and less than the
    # all-depth-first workspace is refused.
    m, n, k = 700, 650, 900
    depth, variant, prec = 2, sm.CLASSIC, sm.PREC_BF16X3
    A = si.normal_f32(31, (m, k))
    B = si.normal_f32(32, (k, n))
    C0 = si.normal_f32(33, (m, n))
    full = sm.strassen_workspace_bytes(m, n, k, depth, variant, prec)
    for t in (1, 2):
        s = sm.make_schedule(strassen_depth=depth, variant=variant, precision=prec, tile=0, split_k=1,
                             strassen_layout=sm.strassen_layout((1 << t) - 1))
        need = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
        assert need < full
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        dC = dev(C0)
        sm.strassen_mm(dev(A), dev(B), dC, depth, variant, prec, workspace=ws)
        torch.cuda.synchronize()
        dC2 = dev(C0)
        sm.semiring_mm(dev(A), dev(B), dC2, sm.PLUS_TIMES, workspace=ws, schedule=s)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().view(np.uint32), dC2.cpu().numpy().view(np.uint32)), t
    with pytest.raises(sm.StarmmError) as e:
        sm.strassen_mm(dev(A), dev(B), dev(C0), depth, variant, prec,
                       workspace=torch.empty(need - 1, dtype=torch.uint8, device="cuda"))
    assert e.value.status == sm.MM_ERR_WORKSPACE


@pytest.mark.parametrize("prec", [sm.PREC_BF16X3, sm.PREC_FP16X3])
def test_star_strassen_over_depth_first_levels_bit_exact(prec):
    # 8-way levels (STAR-Strassen-1) above Strassen levels that are themselves
    # depth-first: every sub-product runs its rounds in turn.
    for (m, n, k) in [(300, 260, 513), (129, 1, 257)]:
        b = exact_bound(sm.WINOGRAD, 2, k)
        g = np.random.default_rng(m + n + k)
        A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
        B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
        C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        s = sm.make_schedule(strassen_depth=2, star_depth=1, variant=sm.WINOGRAD, precision=prec,
                             strassen_layout=sm.strassen_layout(1))
        got = run_schedule(A, B, C0, s)
        assert np.array_equal(got.astype(np.int64), ref), (m, n, k)


@pytest.mark.parametrize("depth,t", [(1, 1), (2, 1), (2, 2)])
def test_strassen_depth_first_full_size_full_matrix(depth, t):
    # n = 8192, classic BF16x3 with t levels depth-first, against the
    # oracle's float64 product on the whole matrix.
    n = 8192
    A, B, ref = _full_size_inputs("normal", n)
    print(f"depth-first Strassen n=8192 depth {depth} t {t}", flush=True)
    s = sm.make_schedule(strassen_depth=depth, variant=sm.CLASSIC, precision=sm.PREC_BF16X3,
                         strassen_layout=sm.strassen_layout((1 << t) - 1))
    got = run_schedule(A, B, np.zeros((n, n), np.float32), s)
    assert np.isfinite(got).all()
    err = oracle.rel_fro(got, ref)
    assert err < tolerance(sm.PREC_BF16X3, sm.CLASSIC, depth, k=n), err
