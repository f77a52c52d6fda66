"""GPU parity of the FP16x3 split-precision product (fp16 hi/lo of operands
scaled per row of A and per column of B by exact powers of two) at depth 0
and under Strassen / Strassen-Winograd levels, against the oracle.

Exactness pins: integer inputs that keep every Strassen operand below 2^8
and every partial sum below 2^24 are exact in the fp16 hi part whatever
power of two scales them (11 significant bits suffice), the lo part is
zero, and the unscaling is exact, so any correct implementation returns
the integer product bit for bit.  At depth 0 the device split must agree
with the oracle's bit-level emulation up to fp32 accumulation.  Rows that
span twelve decades (values that overflow or fall below fp16's normal range
unscaled) must keep a per-row relative error near fp32 accumulation, which
only the scaling makes possible.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

MiB = 1 << 20
PRECS = [sm.PREC_FP16X3, sm.PREC_FP16X3_HIACC]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_strassen(A, B, C0, depth, variant, prec):
    m, k = A.shape
    n = B.shape[1]
    wsb = sm.strassen_workspace_bytes(m, n, k, depth, variant, prec)
    assert wsb > 0
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    dC = dev(C0)
    sm.strassen_mm(dev(A), dev(B), dC, depth, variant, prec, workspace=ws)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def run_semiring(A, B, C0, schedule):
    m, k = A.shape
    n = B.shape[1]
    wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, schedule)
    assert wsb > 0
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    dC = dev(C0)
    sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=schedule)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


def exact_bound(variant, depth, k):
    """Largest integer bound b (inputs in [-b, b]) that keeps every operand
    <= 256 in magnitude and every partial sum below 2^24."""
    growth = (2 if variant == sm.CLASSIC else 4) ** depth
    outputs = 4 ** depth
    leaf_k = -(-k // 2 ** depth)
    b = 8
    while b > 1 and (b * growth > 256 or leaf_k * (b * growth) ** 2 * outputs >= 2 ** 24):
        b //= 2
    return b


def int_case(seed, m, n, k, b):
    g = np.random.default_rng(seed)
    A = g.integers(-b, b + 1, (m, k)).astype(np.float32)
    B = g.integers(-b, b + 1, (k, n)).astype(np.float32)
    C0 = g.integers(-b, b + 1, (m, n)).astype(np.float32)
    # one all-zero row of A and column of B: scale 1, product row / column = C0
    A[m // 2] = 0
    B[:, n // 3] = 0
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    return A, B, C0, ref


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("depth", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", PRECS)
def test_fp16x3_small_integers_bit_exact(variant, depth, prec):
    for (m, n, k) in [(256, 256, 256), (257, 129, 99), (37, 300, 65), (8, 8, 8), (1, 1, 1)]:
        b = exact_bound(variant, depth, k)
        A, B, C0, ref = int_case(m + n + k + depth, m, n, k, b)
        got = run_strassen(A, B, C0, depth, variant, prec)
        assert np.array_equal(got.astype(np.int64), ref), (m, n, k, b)


@pytest.mark.parametrize("depth", [0, 1, 2])
def test_fp16x3_schedules_tile_and_split_exact(depth):
    # FP16x3 through mm_semiring schedules: the (leaf) products take the
    # schedule's tile and k-split, 256 tile included.
    m, n, k = 300, 260, 512
    b = exact_bound(sm.WINOGRAD, depth, k)
    A, B, C0, ref = int_case(depth + 11, m, n, k, b)
    for tile in (32, 64, 128, 256):
        for split in (1, 2, 8):
            s = sm.make_schedule(tile=tile, split_k=split, strassen_depth=depth, variant=sm.WINOGRAD,
                                 precision=sm.PREC_FP16X3)
            got = run_semiring(A, B, C0, s)
            assert np.array_equal(got.astype(np.int64), ref), (tile, split)


@pytest.mark.parametrize("split", [1, 2])
def test_fp16x3_wide_tile_stage_counts_exact(split):
    # The 256-wide planes tile with fp16 operands: k over 1..10 stages of 16
    # (ragged and whole), ragged m and n.
    m, n = 300, 270
    for k in (1, 15, 16, 17, 48, 49, 112, 113, 160):
        A, B, C0, ref = int_case(k, m, n, k, 8)
        s = sm.make_schedule(tile=256, split_k=split, precision=sm.PREC_FP16X3)
        got = run_semiring(A, B, C0, s)
        assert np.array_equal(got.astype(np.int64), ref), (k, split)


def test_fp16x3_split_matches_emulation():
    # Device scales and split (hardware RNE) against the oracle's bit-level
    # binary16 rounding of the scaled operands: only fp32 accumulation and
    # its order remain between the two.
    m, n, k = 96, 80, 512
    A = si.normal_f32(6, (m, k))
    B = si.normal_f32(7, (k, n))
    for tile in (32, 256):
        s = sm.make_schedule(tile=tile, split_k=1, precision=sm.PREC_FP16X3)
        got = run_semiring(A, B, np.zeros((m, n), np.float32), s)
        emu = oracle.split3_fp16_product_f64(A, B)
        assert oracle.rel_fro(got, emu) < 5e-7, tile
        # the split itself: ~2^-22 per product, far below the fp32 accumulation
        assert oracle.rel_fro(got, oracle.fp64_ref(A, B)) < 1e-6, tile


# Relative Frobenius tolerance for N(0,1) inputs: fp32 accumulation over k
# terms (2^-24 sqrt(k) in the typical case) plus the FP16x3 split (7.5e-8
# for this workload in an exact-arithmetic emulation; we allow 2e-7), grown
# by about 2 (classic) or 2.6 (Winograd) per Strassen level.
def tolerance(variant, depth, k=1024):
    base = 2.0 ** -24 * np.sqrt(k) + 2e-7
    growth = 2.0 if variant == sm.CLASSIC else 2.7
    return base * growth ** depth


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
@pytest.mark.parametrize("depth", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", PRECS)
def test_fp16x3_normal_tolerance_and_determinism(variant, depth, prec):
    m, n, k = 1000, 1031, 1024
    A = si.normal_f32(si.BASE_SEED, (m, k))
    B = si.normal_f32(si.BASE_SEED + 1, (k, n))
    C0 = np.zeros((m, n), np.float32)
    got = run_strassen(A, B, C0, depth, variant, prec)
    again = run_strassen(A, B, C0, depth, variant, prec)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    err = oracle.rel_fro(got, oracle.fp64_ref(A, B))
    assert err < tolerance(variant, depth), err


def test_fp16x3_wide_dynamic_range_per_row():
    # Rows of A and columns of B scaled by 10^U(-6, 6): unscaled, such values
    # overflow fp16 (above 65504) or lose their lo part below its normal
    # range.  With the per-row / per-column powers of two every output entry
    # keeps its own relative accuracy (depth 0: no pre-addition mixes rows of
    # different magnitude).
    m, n, k = 384, 320, 512
    A = si.row_scaled_normal_f32(41, (m, k), span=6.0)
    B = si.row_scaled_normal_f32(42, (n, k), span=6.0).T.copy()
    got = run_strassen(A, B, np.zeros((m, n), np.float32), 0, sm.WINOGRAD, sm.PREC_FP16X3)
    assert np.isfinite(got).all()
    ref = oracle.fp64_ref(A, B)
    ra = np.abs(A).max(axis=1)[:, None].astype(np.float64)
    cb = np.abs(B).max(axis=0)[None, :].astype(np.float64)
    err = oracle.rel_fro(got / (ra * cb), ref / (ra * cb))
    assert err < tolerance(sm.WINOGRAD, 0, k), err
    per_row = np.linalg.norm((got - ref) / cb, axis=1) / np.linalg.norm(ref / cb, axis=1)
    assert per_row.max() < 10 * tolerance(sm.WINOGRAD, 0, k), per_row.max()


@pytest.mark.parametrize("depth", [1, 2])
def test_fp16x3_wide_dynamic_range_strassen_normwise(depth):
    # Same data under Strassen-Winograd levels: the pre-additions add rows of
    # different magnitude, so the guarantee is normwise; the scales (taken
    # over the pre-addition's growth) must keep every value finite.
    m, n, k = 384, 320, 512
    A = si.row_scaled_normal_f32(41, (m, k), span=6.0)
    B = si.row_scaled_normal_f32(42, (n, k), span=6.0).T.copy()
    got = run_strassen(A, B, np.zeros((m, n), np.float32), depth, sm.WINOGRAD, sm.PREC_FP16X3)
    assert np.isfinite(got).all()
    err = oracle.rel_fro(got, oracle.fp64_ref(A, B))
    assert err < tolerance(sm.WINOGRAD, depth, k), err


@pytest.mark.parametrize("depth", [1, 2])
@pytest.mark.parametrize("data", ["normal", "rows_scaled"])
def test_fp16x3_full_size_sampled_rows(depth, data):
    # n = 8192 Strassen-Winograd over the FP16x3 base product (256 tiles,
    # direct-to-LDS kernel); sampled rows against the float64 oracle's rows.
    n = 8192
    if data == "normal":
        A = si.normal_f32(si.BASE_SEED, (n, n))
        B = si.normal_f32(si.BASE_SEED + 1, (n, n))
    else:
        A = si.row_scaled_normal_f32(si.BASE_SEED, (n, n))
        B = si.row_scaled_normal_f32(si.BASE_SEED + 1, (n, n))
    got = run_strassen(A, B, np.zeros((n, n), np.float32), depth, sm.WINOGRAD, sm.PREC_FP16X3)
    rows = np.array([0, 1, 1023, 1024, 4095, 4096, 6000, 8191])
    ref = oracle.fp64_rows(A, B, rows)
    err = oracle.rel_fro(got[rows], ref)
    assert err < tolerance(sm.WINOGRAD, depth, k=n), err
    assert np.isfinite(got).all()


def test_fp16x3_and_star_strassen_empty_and_tiny_dimensions():
    # m, n or k = 0 leave C untouched (no launch); k = 1 and 1 x 1 products
    # go through the scale pass and one-stage tiles.
    for (m, n, k) in [(0, 5, 7), (6, 0, 7), (6, 5, 0), (1, 1, 1), (3, 2, 1), (1, 300, 2)]:
        A = si.small_int_f32(50 + m, (m, k))
        B = si.small_int_f32(51 + n, (k, n))
        C0 = si.small_int_f32(52 + k, (m, n))
        ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        for depth, top in ((0, 0), (1, 0), (1, 2)):
            s = sm.make_schedule(strassen_depth=depth, star_depth=top, variant=sm.WINOGRAD, precision=sm.PREC_FP16X3)
            wsb = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
            ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
            dC = dev(C0)
            sm.semiring_mm(dev(A), dev(B), dC, sm.PLUS_TIMES, workspace=ws, schedule=s)
            torch.cuda.synchronize()
            assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref), (m, n, k, depth, top)
