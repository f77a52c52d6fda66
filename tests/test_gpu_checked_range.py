"""GPU parity of the checked-range integer path (MM_FLAG_CHECKED_RANGE):
(min,+) with entries of either sign in [-2^30, 2^30] (2^30 = INF) and (max,+)
in [-2^30, 2^30 - 1] (-2^30 = -INF), bit-exact against the int64 oracle for
every schedule (tile, k-split, TAR/SAR/STAR merge, bands, the persistent
slot ring), at the domain's corners (the most negative sum -2^31, INF times
a negative entry) and on shortest / longest paths with negative weights."""
import math

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

MiB = 1 << 20
INF = sm.INF
CHK = sm.FLAG_CHECKED_RANGE
WIDE = [sm.MIN_PLUS, sm.MAX_PLUS]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.int32)).cuda()


def run(sr, A, B, C0, sched, ws_bytes=0):
    dC = dev(C0)
    ws = torch.zeros(max(ws_bytes, 1), dtype=torch.uint8, device="cuda") if ws_bytes else None
    sm.semiring_mm(dev(A), dev(B), dC, sr, workspace=ws, schedule=sched)
    torch.cuda.synchronize()
    return dC.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("sr", WIDE)
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (33, 65, 17), (129, 255, 300), (300, 200, 1000)])
def test_checked_default_schedule_bit_exact(sr, shape):
    m, n, k = shape
    A = si.wide_i32(sr, 10 + m, (m, k))
    B = si.wide_i32(sr, 11 + n, (k, n))
    C0 = si.wide_i32(sr, 12 + k, (m, n))
    got = run(sr, A, B, C0, sm.make_schedule(flags=CHK), ws_bytes=64 * MiB)
    assert np.array_equal(got, oracle.brute(sr, A, B, C0))


@pytest.mark.parametrize("sr", WIDE)
def test_checked_all_schedules_bit_exact(sr):
    m, n, k = 161, 97, 777
    A = si.wide_i32(sr, 1, (m, k)).astype(np.int64)
    B = si.wide_i32(sr, 2, (k, n)).astype(np.int64)
    # some rows of A and columns of B of one sign only, some rows all sentinel,
    # so that the outputs take both signs and the sentinel
    sgn = 1 if sr == sm.MIN_PLUS else -1
    A[3::7] = sgn * np.abs(A[3::7])
    B[:, ::5] = sgn * np.abs(B[:, ::5])
    A[::11] = sgn * INF
    C0 = si.wide_i32(sr, 3, (m, n), frac_inf=0.3)
    ref = oracle.brute(sr, A, B, C0)
    assert (ref < 0).any() and (ref > 0).any() and (np.abs(ref) == INF).any()
    for tile in (32, 64, 128):
        for s in (1, 2, 8, 64):
            for star in sorted({0, 1, int(np.log2(s))}):
                if star > int(np.log2(s)):
                    continue
                for band in (0, tile):
                    sched = sm.make_schedule(tile=tile, split_k=s, star_depth=star, band_rows=band, flags=CHK)
                    got = run(sr, A, B, C0, sched, ws_bytes=256 * MiB)
                    assert np.array_equal(got, ref), (tile, s, star, band)


@pytest.mark.parametrize("sr", WIDE)
def test_checked_persistent_bit_exact(sr):
    for (m, n, k) in [(1100, 1090, 777), (33, 65, 17), (1, 1, 1)]:
        A = si.wide_i32(sr, m + 1, (m, k))
        B = si.wide_i32(sr, n + 2, (k, n))
        C0 = si.wide_i32(sr, k + 3, (m, n))
        ref = oracle.brute(sr, A, B, C0)
        for tile, split in ((32, 4), (64, 2), (128, 8), (128, 1)):
            sched = sm.make_schedule(tile=tile, split_k=split, flags=sm.FLAG_PERSISTENT | CHK)
            wsb = sm.workspace_bytes(sr, sm.DT_I32, m, n, k, sched)
            got = run(sr, A, B, C0, sched, ws_bytes=wsb)
            assert np.array_equal(got, ref), (m, n, k, tile, split)


def test_checked_domain_corners():
    # (min,+): every entry -2^30 -> every sum is -2^31, the int32 minimum;
    # an INF row of A against negative B stays INF; a sum reaching INF saturates.
    m, n, k = 70, 66, 130
    A = np.full((m, k), -INF, np.int64)
    A[5] = INF
    A[6] = INF - 1
    B = np.full((k, n), -INF, np.int64)
    B[:, 3] = 7  # row 6: (INF - 1) + 7 >= INF
    C0 = np.full((m, n), INF, np.int64)
    for tile, s in ((32, 1), (64, 4), (128, 2)):
        got = run(sm.MIN_PLUS, A, B, C0, sm.make_schedule(tile=tile, split_k=s, flags=CHK), ws_bytes=16 * MiB)
        ref = oracle.brute(sm.MIN_PLUS, A, B, C0)
        assert np.array_equal(got, ref)
        assert got[0, 0] == -2 ** 31 and (got[5] == INF).all() and got[6, 3] == INF and got[6, 0] == INF - 1 - INF
    # (max,+): the largest sum 2^31 - 2; a -INF entry with a positive partner stays -INF
    A = np.full((m, k), INF - 1, np.int64)
    A[5] = -INF
    B = np.full((k, n), INF - 1, np.int64)
    C0 = np.full((m, n), -INF, np.int64)
    got = run(sm.MAX_PLUS, A, B, C0, sm.make_schedule(tile=64, split_k=2, flags=CHK), ws_bytes=16 * MiB)
    assert np.array_equal(got, oracle.brute(sm.MAX_PLUS, A, B, C0))
    assert got[0, 0] == 2 ** 31 - 2 and (got[5] == -INF).all()


@pytest.mark.parametrize("sr", WIDE)
def test_checked_path_closure_with_negative_weights(sr):
    # A DAG with weights of both signs: repeated squaring on the GPU gives the
    # oracle's shortest ((min,+)) / longest ((max,+)) path lengths.
    n = 400
    g = np.random.default_rng(40 + sr)
    W = g.integers(-1000, 1001, (n, n)).astype(np.int64)
    zero = INF if sr == sm.MIN_PLUS else -INF
    W[(g.random((n, n)) < 0.97) | (np.arange(n)[:, None] >= np.arange(n)[None, :])] = zero
    np.fill_diagonal(W, 0)
    D_gpu, D_ref = W.copy(), W.copy()
    for step in range(math.ceil(math.log2(n))):
        sched = sm.make_schedule(tile=(32, 64, 128)[step % 3], split_k=(1, 4, 2)[step % 3], flags=CHK)
        C0 = np.full((n, n), zero, np.int64)
        D_gpu = run(sr, D_gpu, D_gpu, C0, sched, ws_bytes=64 * MiB)
        D_ref = oracle.brute(sr, D_ref, D_ref)
        assert np.array_equal(D_gpu, D_ref), step
    assert ((D_ref < 0) if sr == sm.MIN_PLUS else (D_ref > 0)).any()


def test_checked_full_size_sampled_rows():
    # n = 4096 at the 4x budget (split 4 through temporaries) and with TAR
    # merging; sampled rows bit for bit against the oracle.
    n, sr = 4096, sm.MIN_PLUS
    A = si.wide_i32(sr, si.BASE_SEED, (n, n))
    B = si.wide_i32(sr, si.BASE_SEED + 1, (n, n))
    C0 = si.semiring_init(sr, (n, n))
    rows = np.unique(np.concatenate([[0, 127, 128, 2047, 2048, n - 1], np.random.default_rng(2).integers(0, n, 8)]))
    ref = oracle.brute(sr, A[rows], B, C0[rows])
    for s, star, bx in ((4, 0, 4), (4, 2, 0)):
        sched = sm.make_schedule(tile=128, split_k=s, star_depth=star, flags=CHK)
        got = run(sr, A, B, C0, sched, ws_bytes=bx * n * n * 4)
        assert np.array_equal(got[rows], ref), (s, star)
        assert got.min() >= -2 ** 31 and got.max() <= INF


def test_flag_is_a_no_op_for_maxmin():
    m, n, k = 150, 140, 300
    A = si.maxmin_i32(1, (m, k))
    B = si.maxmin_i32(2, (k, n))
    C0 = si.semiring_init(sm.MAX_MIN, (m, n))
    a = run(sm.MAX_MIN, A, B, C0, sm.make_schedule(tile=64, split_k=2, flags=CHK), ws_bytes=16 * MiB)
    b = run(sm.MAX_MIN, A, B, C0, sm.make_schedule(tile=64, split_k=2), ws_bytes=16 * MiB)
    assert np.array_equal(a, b) and np.array_equal(a, oracle.brute(sm.MAX_MIN, A, B, C0))
