"""GPU parity of one level of a general bilinear scheme (eq. bilinear,
closing remarks of Sec. strassen) over the BF16x3 base product, against the
oracle's level (``oracle.bilinear_ref``).  The schemes are built by the
oracle and handed to the library as coefficient arrays.

Exactness pins: with small-integer inputs every operand sum is an integer
of magnitude <= 256 (exact in bf16, so the lo parts are zero) and every
partial sum stays below 2^24 (exact in fp32), so any correct level returns
the integer product bit for bit.  Normal inputs are held to the split's
error times a growth per scheme (as for Strassen levels: ~2 per classic
level, ~2.7 per Winograd level, ~1 for the definition's own blocks)."""
import numpy as np
import pytest

import oracle
from oracle import bilinear_ref as bl
import synth_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402


def _schemes():
    c = bl.strassen(oracle.STRASSEN_CLASSIC)
    w = bl.strassen(oracle.STRASSEN_WINOGRAD)
    return {  # name: (scheme, error growth)
        "classical2": (bl.classical(2), 1.2), "classical3": (bl.classical(3), 1.2), "classical4": (bl.classical(4), 1.2),
        "strassen": (c, 2.0), "winograd": (w, 2.7), "strassen_x_strassen": (bl.product(c, c), 4.0),
        "winograd_x_classical2": (bl.product(w, bl.classical(2)), 2.7 * 1.2),
    }


def _lib_scheme(s):
    return sm.bilinear_scheme_from_arrays(s.g, s.alpha.tolist(), s.beta.tolist(), s.gamma.tolist())


def run(A, B, C0, scheme):
    m, k = A.shape
    n = B.shape[1]
    ls = _lib_scheme(scheme)
    wsb = sm.bilinear_workspace_bytes(m, n, k, ls)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    dC = torch.from_numpy(np.ascontiguousarray(C0)).cuda()
    sm.bilinear_mm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), dC, ls, workspace=ws)
    torch.cuda.synchronize()
    return dC.cpu().numpy()


@pytest.mark.parametrize("name", list(_schemes()))
@pytest.mark.parametrize("shape", [(1, 1, 1), (33, 17, 65), (130, 257, 190), (512, 384, 640)])
def test_small_integers_bit_exact(name, shape):
    s, _ = _schemes()[name]
    m, n, k = shape
    A = si.small_int_f32(11, (m, k), 2)
    B = si.small_int_f32(12, (k, n), 2)
    C0 = si.small_int_f32(13, (m, n), 2)
    got = run(A, B, C0, s)
    ref = bl.bilinear(A.astype(np.int64), B.astype(np.int64), s, C0.astype(np.int64))
    assert np.array_equal(got.astype(np.int64), ref), (name, shape)


def _tolerance(growth, k):
    return (2.0 ** -24 * np.sqrt(k) + 9e-6) * growth


@pytest.mark.parametrize("name", list(_schemes()))
def test_normal_inputs_within_tolerance_and_deterministic(name):
    s, growth = _schemes()[name]
    m, n, k = 1000, 1031, 1024
    A = si.normal_f32(si.BASE_SEED, (m, k))
    B = si.normal_f32(si.BASE_SEED + 1, (k, n))
    C0 = np.zeros((m, n), np.float32)
    got = run(A, B, C0, s)
    again = run(A, B, C0, s)
    assert np.array_equal(got.view(np.uint32), again.view(np.uint32))
    err = oracle.rel_fro(got, bl.bilinear(A.astype(np.float64), B.astype(np.float64), s))
    assert err < _tolerance(growth, k), (name, err)


@pytest.mark.parametrize("name", ["strassen", "classical3"])
def test_same_bits_for_any_operand_alignment(name):
    # The post-addition updates 16-byte runs of C's rows where a block's
    # columns and C's alignment allow it and single elements elsewhere, and
    # the pre-addition reads A in 16-byte runs under the same condition:
    # operands and C as views at odd offsets give the same bits.
    s, growth = _schemes()[name]
    m, n, k = 300, 1030, 518
    A = si.normal_f32(si.BASE_SEED + 4, (m, k))
    B = si.normal_f32(si.BASE_SEED + 5, (k, n))
    ref = run(A, B, np.zeros((m, n), np.float32), s)
    assert oracle.rel_fro(ref, bl.bilinear(A.astype(np.float64), B.astype(np.float64), s)) < _tolerance(growth, k)
    ls = _lib_scheme(s)
    ws = torch.empty(max(sm.bilinear_workspace_bytes(m, n, k, ls), 1), dtype=torch.uint8, device="cuda")
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for pad, off in ((1, 0), (4, 1), (5, 3)):
        Aw = torch.zeros((m, k + pad), device="cuda")
        Aw[:, off:off + k] = dA
        Bw = torch.zeros((k, n + pad), device="cuda")
        Bw[:, off:off + n] = dB
        Cw = torch.zeros((m, n + pad), device="cuda")
        sm.bilinear_mm(Aw[:, off:off + k], Bw[:, off:off + n], Cw[:, off:off + n], ls, workspace=ws)
        torch.cuda.synchronize()
        got = Cw[:, off:off + n].cpu().numpy()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (pad, off)


def test_accumulates_into_c_and_refuses_a_wrong_scheme():
    s = bl.strassen(oracle.STRASSEN_WINOGRAD)
    m, n, k = 300, 200, 100
    A = si.small_int_f32(21, (m, k), 2)
    B = si.small_int_f32(22, (k, n), 2)
    C0 = si.small_int_f32(23, (m, n), 4)
    got = run(A, B, C0, s)
    assert np.array_equal(got.astype(np.int64), C0.astype(np.int64) + A.astype(np.int64) @ B.astype(np.int64))
    bad = bl.Scheme(s.g, s.alpha.copy(), s.beta.copy(), s.gamma.copy())
    bad.alpha[3, 1] += 1
    with pytest.raises(sm.StarmmError):
        run(A, B, C0, bad)


@pytest.mark.parametrize("name", ["strassen_x_strassen", "classical4"])
def test_full_size_sampled_rows(name):
    # n = 4096, the 4 x 4 grid: 49 (or 64) leaf products of 1024^3 in one
    # launch; every 64th row and the last against the float64 product.
    s, growth = _schemes()[name]
    n = 4096
    A = si.normal_f32(si.BASE_SEED, (n, n))
    B = si.normal_f32(si.BASE_SEED + 1, (n, n))
    got = run(A, B, np.zeros((n, n), np.float32), s)
    rows = np.concatenate([np.arange(0, n, 64), [n - 1]])
    ref = oracle.fp64_rows(A, B, rows)
    assert oracle.rel_fro(got[rows], ref) < _tolerance(growth, n)
