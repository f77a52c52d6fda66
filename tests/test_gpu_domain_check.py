"""GPU: the integer input-domain check (mm_domain_violations) counts exactly
the entries numpy finds outside each semiring's domain, on strided views
too; with STARMM_CHECK_DOMAIN set, mm_semiring refuses operands outside the
domain (C untouched) and runs valid ones to the oracle's result."""
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

INF = sm.INF
CHK = sm.FLAG_CHECKED_RANGE
DOMAINS = [(sm.MIN_PLUS, 0, 0, INF), (sm.MIN_PLUS, CHK, -INF, INF), (sm.MAX_PLUS, 0, -INF, 0),
           (sm.MAX_PLUS, CHK, -INF, INF - 1), (sm.OR_AND, 0, 0, 1), (sm.MAX_MIN, 0, si.I32_MIN, 2 ** 31 - 1)]


@pytest.mark.parametrize("sr,flags,lo,hi", DOMAINS)
def test_counts_match_numpy(sr, flags, lo, hi):
    g = np.random.default_rng(sr * 10 + flags)
    X = g.integers(-2 ** 31, 2 ** 31, (700, 530), dtype=np.int64)
    # most entries inside, some at and just past both ends
    inside = g.integers(max(lo, -2 ** 31), min(hi, 2 ** 31 - 1) + 1, X.shape, dtype=np.int64)
    X = np.where(g.random(X.shape) < 0.9, inside, X)
    X[0, :4] = [lo, hi, max(lo - 1, -2 ** 31), min(hi + 1, 2 ** 31 - 1)]
    X = X.astype(np.int32)
    want = int(((X.astype(np.int64) < lo) | (X.astype(np.int64) > hi)).sum())
    dX = torch.from_numpy(X).cuda()
    assert sm.domain_violations(dX, sr, flags) == want
    view = dX[3:650, 7:500]  # leading dimension 530 > 493 columns
    sub = X[3:650, 7:500].astype(np.int64)
    assert sm.domain_violations(view, sr, flags) == int(((sub < lo) | (sub > hi)).sum())
    assert sm.domain_violations(dX[:0], sr, flags) == 0
    if sr == sm.MAX_MIN:
        assert want == 0
    else:
        assert want > 0


def test_invalid_arguments():
    dX = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(TypeError):
        sm.domain_violations(dX, sm.MIN_PLUS)
    with pytest.raises(sm.StarmmError):
        sm.domain_violations(dX.int(), sm.PLUS_TIMES)
    with pytest.raises(sm.StarmmError):
        sm.domain_violations(dX.int(), sm.MIN_PLUS, flags=64)


def test_check_domain_mode_refuses_and_accepts():
    m, n, k = 300, 260, 410
    A = si.minplus_i32(1, (m, k))
    B = si.minplus_i32(2, (k, n))
    C0 = si.minplus_i32(3, (m, n))
    bad = A.copy()
    bad[17, 33] = -5  # negative: outside the narrow (min,+) domain
    prev = os.environ.get("STARMM_CHECK_DOMAIN")
    os.environ["STARMM_CHECK_DOMAIN"] = "1"
    try:
        dC = torch.from_numpy(C0).cuda()
        with pytest.raises(sm.StarmmError) as ei:
            sm.semiring_mm(torch.from_numpy(bad).cuda(), torch.from_numpy(B).cuda(), dC, sm.MIN_PLUS,
                           schedule=sm.make_schedule(tile=64))
        assert ei.value.status == sm.MM_ERR_INVALID_ARG and "1 entries" in str(ei.value)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy(), C0)  # nothing launched
        # the same operand is inside the checked range
        sm.semiring_mm(torch.from_numpy(bad).cuda(), torch.from_numpy(B).cuda(), dC, sm.MIN_PLUS,
                       schedule=sm.make_schedule(tile=64, flags=CHK))
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), oracle.brute(sm.MIN_PLUS, bad, B, C0))
        dC = torch.from_numpy(C0).cuda()
        sm.semiring_mm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), dC, sm.MIN_PLUS)
        torch.cuda.synchronize()
        assert np.array_equal(dC.cpu().numpy().astype(np.int64), oracle.brute(sm.MIN_PLUS, A, B, C0))
    finally:
        if prev is None:
            del os.environ["STARMM_CHECK_DOMAIN"]
        else:
            os.environ["STARMM_CHECK_DOMAIN"] = prev
