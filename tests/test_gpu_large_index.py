"""Products whose operands hold more than 2^31 elements, so element offsets
of the later rows pass the int32 range: every kernel indexes in 64 bits.
Inputs come from torch's seeded generator on the device (16-17 GB each);
rows past the 2^31-element mark, and the last row, are checked against the
oracle (the integer semiring bit for bit, fp32 within its tolerance)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402

GiB = 1 << 30


def _need(nbytes):
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes + 4 * GiB:
        pytest.skip(f"needs {nbytes / GiB:.1f} GiB of device memory")


def _rows_past_int32(m, k):
    first = (1 << 31) // k + 1  # first row whose start offset exceeds 2^31 elements
    return np.array(sorted({first, first + 1, (first + m) // 2, m - 2, m - 1}))


def test_minplus_rows_past_int32_offsets():
    m, k, n = (1 << 20) + 37, 1 << 12, 40
    _need(m * k * 4)
    g = torch.Generator(device="cuda").manual_seed(1911)
    A = torch.randint(0, 1 << 20, (m, k), dtype=torch.int32, device="cuda", generator=g)
    B = torch.randint(0, 1 << 20, (k, n), dtype=torch.int32, device="cuda", generator=g)
    C = torch.full((m, n), sm.INF, dtype=torch.int32, device="cuda")
    sm.semiring_mm(A, B, C, sm.MIN_PLUS)
    torch.cuda.synchronize()
    rows = _rows_past_int32(m, k)
    sel = torch.from_numpy(rows).cuda()
    Ah = A[sel].cpu().numpy().astype(np.int64)
    ref = oracle.brute(oracle.MIN_PLUS, Ah, B.cpu().numpy().astype(np.int64))
    assert np.array_equal(C[sel].cpu().numpy().astype(np.int64), ref)
    del A, B, C
    torch.cuda.empty_cache()


def test_f32_rows_past_int32_offsets():
    m, k, n = (1 << 19) + 11, 1 << 13, 48
    _need(m * k * 4)
    g = torch.Generator(device="cuda").manual_seed(1912)
    A = torch.randn((m, k), device="cuda", generator=g)
    B = torch.randn((k, n), device="cuda", generator=g)
    C = torch.zeros((m, n), device="cuda")
    sm.semiring_mm(A, B, C, sm.PLUS_TIMES)
    torch.cuda.synchronize()
    rows = _rows_past_int32(m, k)
    sel = torch.from_numpy(rows).cuda()
    ref = oracle.fp64_rows(A[sel].cpu().numpy(), B.cpu().numpy(), np.arange(len(rows)))
    # fp32 accumulation over k terms: 2^-24 sqrt(k) typical, 4x margin
    assert oracle.rel_fro(C[sel].cpu().numpy(), ref) < 4 * 2.0 ** -24 * np.sqrt(k)
    del A, B, C
    torch.cuda.empty_cache()
