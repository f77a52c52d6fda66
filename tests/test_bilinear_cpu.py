"""Host side of the general bilinear level (eq. bilinear, closing remarks of
Sec. strassen), no GPU: the library's built-in schemes and their flat
products against the oracle's own builders, its matrix-multiplication
tensor check against every single-coefficient error, the workspace closed
form, and argument validation."""
import ctypes
import itertools

import numpy as np
import pytest

import oracle
from oracle import bilinear_ref as bl
import paper_1911_05328_amd as sm
from paper_1911_05328_amd import _lib


def _arrays(s):
    g, a, b, c = sm.bilinear_scheme_arrays(s)
    return g, np.array(a), np.array(b), np.array(c)


def _same(lib_s, ref):
    g, a, b, c = _arrays(lib_s)
    return g == ref.g and np.array_equal(a, ref.alpha) and np.array_equal(b, ref.beta) and np.array_equal(c, ref.gamma)


def test_builtin_schemes_equal_the_oracles():
    for g in (1, 2, 3, 4):
        s = sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, g)
        assert _same(s, bl.classical(g)) and sm.bilinear_scheme_ok(s)
    for v in (sm.CLASSIC, sm.WINOGRAD):
        s = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, v)
        assert _same(s, bl.strassen(v)) and sm.bilinear_scheme_ok(s)


def test_flat_products_equal_the_oracles():
    c2 = sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, 2)
    st = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
    wi = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.WINOGRAD)
    rc2, rst, rwi = bl.classical(2), bl.strassen(oracle.STRASSEN_CLASSIC), bl.strassen(oracle.STRASSEN_WINOGRAD)
    for (x, rx), (y, ry) in itertools.product([(c2, rc2), (st, rst), (wi, rwi)], repeat=2):
        p = sm.bilinear_scheme_product(x, y)
        assert _same(p, bl.product(rx, ry))
        assert sm.bilinear_scheme_ok(p)


def test_product_limits():
    c2 = sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, 2)
    c3 = sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, 3)
    with pytest.raises(sm.StarmmError):
        sm.bilinear_scheme_product(c2, c3)  # 6 x 6 grid
    st = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
    ss = sm.bilinear_scheme_product(st, st)
    assert sm.bilinear_scheme_product(ss, sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, 1)).products == 49
    with pytest.raises(sm.StarmmError):
        sm.bilinear_scheme_product(ss, c2)  # 8 x 8 grid, 392 products
    for bad in ((sm.BILINEAR_CLASSICAL, 0), (sm.BILINEAR_CLASSICAL, 5), (sm.BILINEAR_STRASSEN, 7), (9, 1)):
        with pytest.raises(sm.StarmmError):
            sm.bilinear_scheme(*bad)


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
def test_check_rejects_every_single_wrong_coefficient(variant):
    s = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, variant)
    g, a, b, c = _arrays(s)
    for name, arr in (("alpha", a), ("beta", b), ("gamma", c)):
        for idx in itertools.product(*(range(d) for d in arr.shape)):
            for delta in (-1, 1):
                aa, bb, cc = a.copy(), b.copy(), c.copy()
                {"alpha": aa, "beta": bb, "gamma": cc}[name][idx] += delta
                bad = sm.bilinear_scheme_from_arrays(g, aa, bb, cc)
                assert not sm.bilinear_scheme_ok(bad), (name, idx, delta)
                assert not bl.is_mm(bl.Scheme(g, aa, bb, cc))


def test_workspace_closed_form():
    def r32(x):
        return -(-x // 32) * 32

    def rk(x):  # plane row length: k rounded up to the 32-deep k-step of the bf16 tiles
        return -(-max(x, 1) // 32) * 32

    def r256(x):
        return -(-x // 256) * 256
    for kind, param in ((sm.BILINEAR_STRASSEN, sm.CLASSIC), (sm.BILINEAR_CLASSICAL, 3), (sm.BILINEAR_CLASSICAL, 4)):
        s = sm.bilinear_scheme(kind, param)
        g, R = s.g, s.products
        for m, n, k in ((8192, 8192, 8192), (1000, 999, 77), (5, 3, 2)):
            hm, hk, hn = -(-m // g), -(-k // g), -(-n // g)
            lpk = rk(hk)
            want = r256(r256(R * 2 * r32(hm) * lpk * 2) + R * 2 * r32(hn) * lpk * 2)
            want = r256(want + R * hm * (-(-hn // 4) * 4) * 4)
            assert sm.bilinear_workspace_bytes(m, n, k, s) == want, (kind, param, m, n, k)
    s = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
    assert sm.bilinear_workspace_bytes(8192, 8192, 8192, s) == \
        sm.strassen_workspace_bytes(8192, 8192, 8192, 1, sm.CLASSIC, sm.PREC_BF16X3)
    assert sm.bilinear_workspace_bytes(0, 64, 64, s) == 0
    assert sm.bilinear_workspace_bytes(64, 64, 64, s, sm.PREC_F32) == 0


def test_argument_validation_before_any_launch():
    L = _lib.lib()
    P = ctypes.c_void_p(4096)
    s = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
    # empty products launch nothing
    assert L.mm_bilinear(0, 16, 16, P, 16, P, 16, P, 16, ctypes.byref(s), sm.PREC_BF16X3, None, 0, None) == sm.MM_OK
    # unsupported precision, bad scheme, bad shapes, short workspace
    assert L.mm_bilinear(16, 16, 16, P, 16, P, 16, P, 16, ctypes.byref(s), sm.PREC_F32, None, 0,
                         None) == sm.MM_ERR_UNSUPPORTED
    bad = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
    bad.gamma[0] = -bad.gamma[0]
    assert L.mm_bilinear(16, 16, 16, P, 16, P, 16, P, 16, ctypes.byref(bad), sm.PREC_BF16X3, None, 0,
                         None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_bilinear(16, 16, 16, P, 8, P, 16, P, 16, ctypes.byref(s), sm.PREC_BF16X3, None, 0,
                         None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_bilinear(16, 16, 16, None, 16, P, 16, P, 16, ctypes.byref(s), sm.PREC_BF16X3, None, 0,
                         None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_bilinear(16, 16, 16, P, 16, P, 16, P, 16, ctypes.byref(s), sm.PREC_BF16X3, P, 100,
                         None) == sm.MM_ERR_WORKSPACE
    zero = _lib.BilinearScheme()
    assert L.mm_bilinear_scheme_check(ctypes.byref(zero)) == sm.MM_ERR_INVALID_ARG
