"""GPU parity of mm_semiring against the oracle.

(min,+) / (max,+) / (max, min) / Boolean int32: bit-exact against the int64
oracle for every schedule (tile, k-split, TAR/SAR/STAR merge, bands).  fp32 (+,x) on MFMA:
bit-exact on small-integer inputs (every partial sum is an integer below
2^24, so any summation order gives the same float), and within a relative
Frobenius tolerance on random inputs.
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


def run_semiring(sr, A, B, C0, sched=None, ws_bytes=0):
    dA, dB, dC = dev(A), dev(B), dev(C0)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda") if ws_bytes else None
    sm.semiring_mm(dA, dB, dC, sr, workspace=ws, schedule=sched)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


SHAPES = [(1, 1, 1), (5, 7, 3), (33, 65, 17), (128, 128, 128), (129, 255, 300), (300, 200, 1000)]
INT_SEMIRINGS = [sm.MIN_PLUS, sm.MAX_PLUS, sm.MAX_MIN, sm.OR_AND]


def operand(sr, seed, shape, k):
    """Semiring operand; Boolean ones get density 1/sqrt(k), so that about
    63% of the outputs are true rather than all of them."""
    if sr == sm.OR_AND:
        return si.bool_i32(seed, shape, min(0.5, 1.0 / np.sqrt(max(k, 1))))
    return si.semiring_operand(sr, seed, shape)


@pytest.mark.parametrize("sr", INT_SEMIRINGS)
@pytest.mark.parametrize("shape", SHAPES)
def test_semiring_default_schedule_bit_exact(sr, shape):
    m, n, k = shape
    A = operand(sr, 10 + m, (m, k), k)
    B = operand(sr, 11 + n, (k, n), k)
    C0 = si.semiring_operand(sr, 12 + k, (m, n)) if sr != sm.OR_AND else si.bool_i32(12 + k, (m, n), 0.2)
    ref = oracle.brute(sr, A, B, C0)
    got = run_semiring(sr, A, B, C0, ws_bytes=64 * MiB)
    assert np.array_equal(got.astype(np.int64), ref)


@pytest.mark.parametrize("sr", INT_SEMIRINGS)
def test_semiring_all_schedules_bit_exact(sr):
    m, n, k = 161, 97, 777
    A = operand(sr, 1, (m, k), k)
    B = operand(sr, 2, (k, n), k)
    C0 = si.semiring_init(sr, (m, n))
    ref = oracle.brute(sr, A, B, C0)
    for tile in (32, 64, 128):
        for s in (1, 2, 4, 8, 64):
            for star in sorted({0, 1, int(np.log2(s))}):
                if star > int(np.log2(s)):
                    continue
                for band in (0, tile):
                    sched = sm.make_schedule(tile=tile, split_k=s, star_depth=star, band_rows=band)
                    got = run_semiring(sr, A, B, C0, sched, ws_bytes=256 * MiB)
                    assert np.array_equal(got.astype(np.int64), ref), (tile, s, star, band)


def test_semiring_strided_operands():
    sr = sm.MIN_PLUS
    m, n, k = 70, 90, 130
    Abig = si.minplus_i32(3, (m, k + 7))
    Bbig = si.minplus_i32(4, (k, n + 5))
    A, B = Abig[:, :k], Bbig[:, :n]
    C0 = si.semiring_init(sr, (m, n))
    ref = oracle.brute(sr, A, B, C0)
    dA, dB = dev(Abig)[:, :k], dev(Bbig)[:, :n]
    dC = dev(C0)
    sm.semiring_mm(dA, dB, dC, sr, schedule=sm.make_schedule(tile=32, split_k=2, star_depth=1))
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy().astype(np.int64), ref)


def test_semiring_degenerate_cases():
    sr = sm.MIN_PLUS
    # all-INF operand: C unchanged
    A = np.full((64, 64), sm.INF, dtype=np.int32)
    B = si.minplus_i32(5, (64, 64))
    C0 = si.minplus_i32(6, (64, 64))
    assert np.array_equal(run_semiring(sr, A, B, C0), C0)
    # identity of the semiring
    I = np.full((64, 64), sm.INF, dtype=np.int32)
    np.fill_diagonal(I, 0)
    C0 = si.semiring_init(sr, (64, 64))
    assert np.array_equal(run_semiring(sr, I, B, C0), B)
    # INF + INF saturates (no int32 wrap)
    A = np.full((8, 8), sm.INF, dtype=np.int32)
    assert (run_semiring(sr, A, A, C0[:8, :8].copy()) == sm.INF).all()
    # k = 0 leaves C unchanged; m = 0 is a no-op
    C1 = si.minplus_i32(7, (16, 16))
    dA = torch.empty((16, 0), dtype=torch.int32, device="cuda")
    dB = torch.empty((0, 16), dtype=torch.int32, device="cuda")
    dC = dev(C1)
    sm.semiring_mm(dA, dB, dC, sr)
    torch.cuda.synchronize()
    assert np.array_equal(dC.cpu().numpy(), C1)


@pytest.mark.parametrize("sr", [sm.MAX_MIN, sm.OR_AND])
def test_semiring_identity_and_zero_operand(sr):
    # identity (the semiring's one on the diagonal, zero elsewhere) and an
    # all-zero operand, for (max, min) and Boolean
    n = 96
    one, zero = (si.I32_MAX, si.I32_MIN) if sr == sm.MAX_MIN else (1, 0)
    I = np.full((n, n), zero, dtype=np.int32)
    np.fill_diagonal(I, one)
    B = operand(sr, 8, (n, n), n)
    for sched in (None, sm.make_schedule(tile=32, split_k=4, star_depth=1)):
        assert np.array_equal(run_semiring(sr, I, B, si.semiring_init(sr, (n, n)), sched, 64 * MiB), B)
        Z = np.full((n, n), zero, dtype=np.int32)
        C0 = operand(sr, 9, (n, n), n)
        assert np.array_equal(run_semiring(sr, Z, B, C0, sched, 64 * MiB), C0)


@pytest.mark.parametrize("sr,budget_x,s,star", [
    (sr, bx, s, st) for sr in (sm.MIN_PLUS, sm.MAX_PLUS)
    for bx, s, st in [(0, 1, 0), (1, 2, 0), (2, 2, 0), (4, 4, 0), (0, 4, 2), (1, 4, 1)]] + [
    (sr, bx, s, st) for sr in (sm.MAX_MIN, sm.OR_AND) for bx, s, st in [(0, 1, 0), (2, 2, 0), (0, 4, 2)]])
def test_semiring_full_size_sampled_rows(sr, budget_x, s, star):
    # n = 4096 with 10 % INF entries, at the workspace budgets 0/1x/2x/4x n^2
    # int32; sampled output rows (incl. first/last and band edges) are
    # compared bit for bit with the oracle's rows.
    n = 4096
    A = operand(sr, si.BASE_SEED, (n, n), n)
    B = operand(sr, si.BASE_SEED + 1, (n, n), n)
    C0 = si.semiring_init(sr, (n, n))
    sched = sm.make_schedule(tile=128, split_k=s, star_depth=star)
    got = run_semiring(sr, A, B, C0, sched, ws_bytes=budget_x * n * n * 4)
    rows = np.unique(np.concatenate([[0, 127, 128, 1365, 2047, 2048, n - 1],
                                     np.random.default_rng(0).integers(0, n, 9)]))
    ref = oracle.brute(sr, A[rows], B, C0[rows])
    assert np.array_equal(got[rows].astype(np.int64), ref)
    # whole-matrix properties: within the domain, saturated exactly at the sentinel
    if sr == sm.MIN_PLUS:
        assert got.min() >= 0 and got.max() <= sm.INF
    elif sr == sm.MAX_PLUS:
        assert got.max() <= 0 and got.min() >= -sm.INF
    elif sr == sm.OR_AND:
        assert set(np.unique(got).tolist()) <= {0, 1}
    else:  # (max, min) returns entries of its operands (or the zero)
        assert np.isin(got[rows[:4]], np.concatenate([A[rows[:4]].ravel(), B.ravel(), [si.I32_MIN]])).all()


def test_minplus_full_matrix_against_oracle_every_budget():
    # n = 4096 (min,+) with 10 % INF: the whole C of the budget-4x schedule
    # (k split 4, three temporaries) against the oracle's brute force, element
    # by element; then the whole C of every other budget and merge form
    # against that result (every tile row and XCD range is covered).
    sr, n = sm.MIN_PLUS, 4096
    A = si.minplus_i32(si.BASE_SEED, (n, n))
    B = si.minplus_i32(si.BASE_SEED + 1, (n, n))
    C0 = si.semiring_init(sr, (n, n))
    print("full-matrix (min,+) n=4096: GPU budget 4x", flush=True)
    got4 = run_semiring(sr, A, B, C0, sm.make_schedule(tile=128, split_k=4), ws_bytes=4 * n * n * 4)
    print("full-matrix (min,+) n=4096: oracle", flush=True)
    ref = oracle.brute(sr, A, B, C0)
    assert np.array_equal(got4.astype(np.int64), ref)
    for budget_x, sched in ((0, sm.make_schedule(tile=128, split_k=1)),
                            (1, sm.make_schedule(tile=128, split_k=2)),
                            (2, sm.make_schedule(tile=128, split_k=2)),
                            (0, sm.make_schedule(tile=128, split_k=4, star_depth=2)),
                            (0, sm.make_schedule(tile=64, split_k=16, star_depth=1, band_rows=512)),
                            (None, sm.make_schedule(tile=128, split_k=4, flags=sm.FLAG_PERSISTENT))):
        print(f"full-matrix (min,+) n=4096: budget {budget_x} schedule {sched.as_dict()}", flush=True)
        if budget_x is None:
            ws_bytes = sm.workspace_bytes(sr, sm.DT_I32, n, n, n, sched)
        else:
            ws_bytes = budget_x * n * n * 4 if budget_x else (
                sm.workspace_bytes(sr, sm.DT_I32, n, n, n, sched) or 0)
        got = run_semiring(sr, A, B, C0, sched, ws_bytes=ws_bytes)
        assert np.array_equal(got, got4), sched.as_dict()


# ------------------------------------------------------------------ fp32 MFMA


def run_f32(A, B, C0, sched=None, ws_bytes=0):
    dA, dB, dC = dev(A), dev(B), dev(C0)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda") if ws_bytes else None
    sm.semiring_mm(dA, dB, dC, sm.PLUS_TIMES, workspace=ws, schedule=sched)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


@pytest.mark.parametrize("shape", [(1, 1, 1), (31, 33, 35), (128, 128, 128), (257, 129, 511), (1000, 520, 1024)])
def test_f32_small_integers_bit_exact(shape):
    m, n, k = shape
    A = si.small_int_f32(1, (m, k))
    B = si.small_int_f32(2, (k, n))
    C0 = si.small_int_f32(3, (m, n))
    ref = oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
    for tile in (32, 64, 128):
        for s in (1, 4):
            got = run_f32(A, B, C0, sm.make_schedule(tile=tile, split_k=s), ws_bytes=64 * MiB)
            assert np.array_equal(got.astype(np.int64), ref), (tile, s)


def test_f32_plain_dc_n256_tolerance():
    # Plain 8-way D&C, n = 256, base tile 32, U[-1, 1], no split: rel. Frobenius
    # error vs the float64 oracle below 1e-6 (fp32 accumulation over k = 256).
    n = 256
    A = si.uniform_f32(si.BASE_SEED, (n, n))
    B = si.uniform_f32(si.BASE_SEED + 1, (n, n))
    C0 = np.zeros((n, n), np.float32)
    got = run_f32(A, B, C0, sm.make_schedule(tile=32, split_k=1))
    ref = oracle.rec8(oracle.PLUS_TIMES, A.astype(np.float64), B.astype(np.float64), b=32)
    assert oracle.rel_fro(got, ref) < 1e-6


def test_f32_split_k_deterministic():
    m, n, k = 300, 260, 4096
    A = si.uniform_f32(5, (m, k))
    B = si.uniform_f32(6, (k, n))
    C0 = si.uniform_f32(7, (m, n))
    sched = sm.make_schedule(tile=64, split_k=8)
    a = run_f32(A, B, C0, sched, ws_bytes=64 * MiB)
    b = run_f32(A, B, C0, sched, ws_bytes=64 * MiB)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    ref = oracle.fp64_ref(A, B, C0)
    assert oracle.rel_fro(a, ref) < 2e-6


def test_f32_full_size_full_matrix():
    # The plain D&C fp32 kernel at n = 8192 (the comparison baseline),
    # against the oracle's float64 product on the whole matrix; also every
    # row on its own (no tile row or XCD range hides behind the norm).
    n = 8192
    A = si.normal_f32(si.BASE_SEED, (n, n))
    B = si.normal_f32(si.BASE_SEED + 1, (n, n))
    C0 = np.zeros((n, n), np.float32)
    got = run_f32(A, B, C0, sm.make_schedule(tile=128, split_k=1))
    ref = oracle.fp64_ref(A, B)
    assert oracle.rel_fro(got, ref) < 2e-6
    assert oracle.row_rel_err(got, ref).max() < 4e-6


def run_persistent(sr, A, B, C0, tile, split):
    m, k = A.shape
    n = B.shape[1]
    sched = sm.make_schedule(tile=tile, split_k=split, flags=sm.FLAG_PERSISTENT)
    wsb = sm.workspace_bytes(sr, sm.DT_I32, m, n, k, sched)
    ws = torch.zeros(wsb, dtype=torch.uint8, device="cuda")
    dC = dev(C0)
    sm.semiring_mm(dev(A), dev(B), dC, sr, workspace=ws, schedule=sched, check_persistent=False)
    torch.cuda.synchronize()
    # no bounded wait gave up (mm_persistent_status reads the control block's
    # error word), and the word itself is 0
    sm.persistent_status(ws)
    err = int(ws[8:12].cpu().numpy().view(np.uint32)[0])
    return dC.cpu().numpy(), err


@pytest.mark.parametrize("sr", INT_SEMIRINGS)
def test_persistent_slot_ring_bit_exact(sr):
    # Far more tiles than slot groups (1225 tiles of 32 against 512 groups
    # at split 4, 32 groups at split 64), so every group is reused; ragged
    # edges; split 1 uses no slots.
    for (m, n, k) in [(1100, 1090, 777), (33, 65, 17), (1, 1, 1), (300, 200, 1000)]:
        A = operand(sr, m + 1, (m, k), k)
        B = operand(sr, n + 2, (k, n), k)
        C0 = si.semiring_operand(sr, k + 3, (m, n)) if sr != sm.OR_AND else si.bool_i32(k + 3, (m, n), 0.2)
        ref = oracle.brute(sr, A, B, C0)
        for tile, split in ((32, 4), (32, 64), (64, 2), (128, 8), (128, 1)):
            got, err = run_persistent(sr, A, B, C0, tile, split)
            assert err == 0
            assert np.array_equal(got.astype(np.int64), ref), (m, n, k, tile, split)


@pytest.mark.parametrize("tile,split", [(128, 4), (64, 16)])
def test_persistent_full_size_sampled_rows(tile, split):
    # n = 4096 (min,+) with 10 % INF in one persistent launch; the slot ring
    # holds 2048 tiles whatever n is.
    sr, n = sm.MIN_PLUS, 4096
    A = si.semiring_operand(sr, si.BASE_SEED, (n, n))
    B = si.semiring_operand(sr, si.BASE_SEED + 1, (n, n))
    C0 = si.semiring_init(sr, (n, n))
    got, err = run_persistent(sr, A, B, C0, tile, split)
    assert err == 0
    rows = np.unique(np.concatenate([[0, 127, 128, 2047, 2048, n - 1], np.random.default_rng(1).integers(0, n, 8)]))
    ref = oracle.brute(sr, A[rows], B, C0[rows])
    assert np.array_equal(got[rows].astype(np.int64), ref)


def test_persistent_more_slices_than_k_tiles():
    # split 64 with k = 20 (two 16-deep k-tiles): most slices are empty and
    # contribute the semiring zero; every tile still merges exactly once.
    sr = sm.MIN_PLUS
    m, n, k = 300, 170, 20
    A = si.minplus_i32(61, (m, k))
    B = si.minplus_i32(62, (k, n))
    C0 = si.minplus_i32(63, (m, n))
    ref = oracle.brute(sr, A, B, C0)
    for tile in (32, 128):
        got, err = run_persistent(sr, A, B, C0, tile, 64)
        assert err == 0
        assert np.array_equal(got.astype(np.int64), ref), tile


@pytest.mark.parametrize("sr", [sm.MIN_PLUS, sm.MAX_MIN])
def test_rectangular_shapes_against_largest_dimension_recursion(sr):
    # Tall, wide and deep products (rectangular tile grids walked along their
    # long side, deep k split by the planner) against the oracle's recursion
    # that halves the largest dimension.
    for (m, n, k) in [(4096, 64, 300), (64, 4096, 300), (100, 130, 20000)]:
        A = si.semiring_operand(sr, m + 5, (m, k))
        B = si.semiring_operand(sr, n + 6, (k, n))
        C0 = si.semiring_init(sr, (m, n))
        ref = oracle.rec_rect(sr, A, B, C0, b=64)
        for sched in (None, sm.make_schedule(tile=32, split_k=1), sm.make_schedule(tile=128, split_k=8)):
            got = run_semiring(sr, A, B, C0, sched, ws_bytes=256 * MiB)
            assert np.array_equal(got.astype(np.int64), ref), (m, n, k)


@pytest.mark.parametrize("prec", [sm.PREC_F32, sm.PREC_BF16X3])
def test_f32_tar_atomic_merge_tolerance(prec):
    # TAR levels on floats (MM_FLAG_NONDETERMINISTIC): the k-slices of a
    # group are added into C by atomics in arrival order, so bits may vary
    # run to run; the error stays that of the same product with temporaries.
    m, n, k = 700, 650, 3000
    A = si.normal_f32(71, (m, k))
    B = si.normal_f32(72, (k, n))
    C0 = si.normal_f32(73, (m, n))
    ref = oracle.fp64_ref(A, B, C0)
    tol = 2.0 ** -24 * np.sqrt(k) * 4 if prec == sm.PREC_F32 else 2e-5
    for s, star in ((4, 2), (8, 1), (16, 4)):
        sched = sm.make_schedule(tile=64, split_k=s, star_depth=star, precision=prec, band_rows=m,
                                 flags=sm.FLAG_NONDETERMINISTIC)
        got = run_f32(A, B, C0, sched, ws_bytes=64 * MiB)
        assert oracle.rel_fro(got, ref) < tol, (s, star)
