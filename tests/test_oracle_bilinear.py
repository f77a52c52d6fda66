"""Pins of the oracle's bilinear-scheme level (eq. bilinear, closing remarks
of Sec. strassen) against what mathematics fixes, not against itself:

* every built scheme reproduces the 2 x 2 x 2 (or g x g x g) matrix
  multiplication tensor, checked entry by entry (``is_mm``), and that check
  catches every single wrong coefficient of a seven-product scheme;
* over Z the level equals the library product ``A @ B`` exactly, on ragged
  sizes (zero padding is exact over a ring);
* the flat product scheme Strassen x Strassen (4 x 4 grid, 49 products)
  equals two levels of the oracle's recursive Strassen exactly;
* on float64 data the level stays within a small multiple of the
  classical product's rounding.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import bilinear_ref as bl


def _schemes():
    s_c = bl.strassen(oracle.STRASSEN_CLASSIC)
    s_w = bl.strassen(oracle.STRASSEN_WINOGRAD)
    return {
        "classical2": bl.classical(2), "classical3": bl.classical(3), "classical4": bl.classical(4),
        "strassen": s_c, "winograd": s_w,
        "strassen_x_strassen": bl.product(s_c, s_c),
        "winograd_x_classical2": bl.product(s_w, bl.classical(2)),
        "classical2_x_strassen": bl.product(bl.classical(2), s_c),
    }


@pytest.mark.parametrize("name", list(_schemes()))
def test_schemes_reproduce_the_mm_tensor(name):
    s = _schemes()[name]
    assert bl.is_mm(s), name
    # sizes: g^3 products for the definition, 7 per Strassen factor
    expect = {"classical2": 8, "classical3": 27, "classical4": 64, "strassen": 7, "winograd": 7,
              "strassen_x_strassen": 49, "winograd_x_classical2": 56, "classical2_x_strassen": 56}
    assert s.products == expect[name]


@pytest.mark.parametrize("variant", [oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD])
def test_tensor_check_catches_every_single_wrong_coefficient(variant):
    s = bl.strassen(variant)
    for arr_name in ("alpha", "beta", "gamma"):
        arr = getattr(s, arr_name)
        for idx in itertools.product(*(range(d) for d in arr.shape)):
            for delta in (-1, 1):
                bad = bl.Scheme(s.g, s.alpha.copy(), s.beta.copy(), s.gamma.copy())
                getattr(bad, arr_name)[idx] += delta
                assert not bl.is_mm(bad), (arr_name, idx, delta)


@pytest.mark.parametrize("name", list(_schemes()))
def test_level_exact_over_z_on_ragged_sizes(name):
    s = _schemes()[name]
    g = np.random.default_rng(3)
    for _ in range(6):
        m, n, k = (int(x) for x in g.integers(1, 41, 3))
        A = g.integers(-50, 51, (m, k))
        B = g.integers(-50, 51, (k, n))
        C0 = g.integers(-50, 51, (m, n))
        assert np.array_equal(bl.bilinear(A, B, s, C0), C0 + A @ B), (name, m, n, k)


def test_wrong_scheme_gives_a_wrong_product():
    s = bl.strassen(oracle.STRASSEN_CLASSIC)
    bad = bl.Scheme(s.g, s.alpha.copy(), s.beta.copy(), s.gamma.copy())
    bad.gamma[0, 0] = -bad.gamma[0, 0]
    A = np.arange(16).reshape(4, 4)
    B = np.arange(16).reshape(4, 4)[::-1].copy()
    assert not np.array_equal(bl.bilinear(A, B, bad), A @ B)


@pytest.mark.parametrize("variant", [oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD])
def test_flat_product_scheme_equals_two_recursive_levels(variant):
    s = bl.strassen(variant)
    ss = bl.product(s, s)
    g = np.random.default_rng(4)
    for n in (4, 8, 20, 36):
        A = g.integers(-30, 31, (n, n))
        B = g.integers(-30, 31, (n, n))
        two = oracle.strassen(A, B, depth=2, variant=variant)
        assert np.array_equal(bl.bilinear(A, B, ss), two), n


@pytest.mark.parametrize("name", ["strassen", "winograd", "classical3", "strassen_x_strassen"])
def test_float64_level_close_to_classical(name):
    s = _schemes()[name]
    g = np.random.default_rng(5)
    A = g.standard_normal((96, 80))
    B = g.standard_normal((80, 72))
    R = A @ B
    assert oracle.rel_fro(bl.bilinear(A, B, s), R) < 1e-13
