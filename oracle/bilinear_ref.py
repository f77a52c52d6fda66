"""Oracle: one level of a bilinear matrix-multiplication scheme.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this module; the product library
never imports it and shares no code with it.

The closing remarks of Sec. strassen (eq. bilinear) write every
Strassen-like algorithm as a bilinear circuit: each output block C_i is a sum
over products, each product multiplying a signed combination of blocks of A
by a signed combination of blocks of B, with constant coefficients.  Here a
scheme on a g x g block grid with R products is three integer arrays:

* ``alpha`` (R x g*g): the A-side operand of product r is
  S_r = sum_p alpha[r, p] A_p, block p = i*g + l in block-row i and
  block-column l of A;
* ``beta``  (R x g*g): T_r = sum_q beta[r, q] B_q, block q = l*g + j of B;
* ``gamma`` (g*g x R): C_c gains sum_r gamma[c, r] (S_r T_r), block
  c = i*g + j of C.

It multiplies matrices exactly when its coefficients reproduce the matrix
multiplication tensor: sum_r alpha[r, (i, l)] beta[r, (l', j)] gamma[(i', j'), r]
is 1 if i = i', l = l', j = j' and 0 otherwise (``is_mm``).

Builders: ``classical(g)`` (the g^3 block products of the definition),
``strassen(variant)`` (the 2 x 2 schemes the oracle's Strassen uses, as
printed in Sec. strassen or Strassen-Winograd), and ``product(s1, s2)``: the
scheme on the (g1 g2) x (g1 g2) grid whose products are the pairs of
products of s1 and s2 (one flat level doing what s1 over s2 does in two).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import _SW_CLASSIC, _SW_WINOGRAD, STRASSEN_CLASSIC


class Scheme:
    """A bilinear scheme: grid g, coefficient arrays alpha, beta, gamma."""

    def __init__(self, g: int, alpha, beta, gamma):
        self.g = int(g)
        self.alpha = np.asarray(alpha, dtype=np.int64)
        self.beta = np.asarray(beta, dtype=np.int64)
        self.gamma = np.asarray(gamma, dtype=np.int64)
        R = self.alpha.shape[0]
        gg = self.g * self.g
        assert self.alpha.shape == (R, gg) and self.beta.shape == (R, gg) and self.gamma.shape == (gg, R)

    @property
    def products(self) -> int:
        return self.alpha.shape[0]


def classical(g: int) -> Scheme:
    """The definition itself on a g x g grid: product (i, l, j) is
    A_{il} B_{lj}, added into C_{ij}."""
    R = g ** 3
    alpha = np.zeros((R, g * g), dtype=np.int64)
    beta = np.zeros((R, g * g), dtype=np.int64)
    gamma = np.zeros((g * g, R), dtype=np.int64)
    for r, (i, l, j) in enumerate(itertools.product(range(g), repeat=3)):
        alpha[r, i * g + l] = 1
        beta[r, l * g + j] = 1
        gamma[i * g + j, r] = 1
    return Scheme(g, alpha, beta, gamma)


def strassen(variant: int = STRASSEN_CLASSIC) -> Scheme:
    """The seven-product 2 x 2 scheme of the oracle's Strassen (quadrant
    q = 2 * row + column for A, B and C alike)."""
    table = _SW_CLASSIC if variant == STRASSEN_CLASSIC else _SW_WINOGRAD
    alpha = np.zeros((7, 4), dtype=np.int64)
    beta = np.zeros((7, 4), dtype=np.int64)
    gamma = np.zeros((4, 7), dtype=np.int64)
    for r, (sa, sb, sc) in enumerate(table):
        for q, c in sa.items():
            alpha[r, q] = c
        for q, c in sb.items():
            beta[r, q] = c
        for q, c in sc.items():
            gamma[q, r] = c
    return Scheme(2, alpha, beta, gamma)


def product(s1: Scheme, s2: Scheme) -> Scheme:
    """s1 applied to the g1 x g1 grid of blocks, s2 inside each block, as one
    level on the g1 g2 x g1 g2 grid: block index i = i1 g2 + i2 (coarse i1,
    fine i2), product r = r1 R2 + r2, coefficients multiplied."""
    g1, g2 = s1.g, s2.g
    g = g1 * g2
    R1, R2 = s1.products, s2.products
    alpha = np.zeros((R1 * R2, g * g), dtype=np.int64)
    beta = np.zeros((R1 * R2, g * g), dtype=np.int64)
    gamma = np.zeros((g * g, R1 * R2), dtype=np.int64)

    def fine(b1, b2, gg1, gg2):
        """flat block index of fine block b2 inside coarse block b1"""
        i1, l1 = divmod(b1, gg1)
        i2, l2 = divmod(b2, gg2)
        return (i1 * gg2 + i2) * (gg1 * gg2) + (l1 * gg2 + l2)

    for r1, r2 in itertools.product(range(R1), range(R2)):
        r = r1 * R2 + r2
        for b1, b2 in itertools.product(range(g1 * g1), range(g2 * g2)):
            f = fine(b1, b2, g1, g2)
            alpha[r, f] = s1.alpha[r1, b1] * s2.alpha[r2, b2]
            beta[r, f] = s1.beta[r1, b1] * s2.beta[r2, b2]
            gamma[f, r] = s1.gamma[b1, r1] * s2.gamma[b2, r2]
    return Scheme(g, alpha, beta, gamma)


def is_mm(s: Scheme) -> bool:
    """Whether the scheme reproduces the matrix multiplication tensor on its
    grid (every one of the g^6 index combinations checked)."""
    g = s.g
    for i, l, lp, j, ip, jp in itertools.product(range(g), repeat=6):
        t = int(np.sum(s.alpha[:, i * g + l] * s.beta[:, lp * g + j] * s.gamma[ip * g + jp, :]))
        want = 1 if (i == ip and l == lp and j == jp) else 0
        if t != want:
            return False
    return True


def _blocks(X, g):
    """The g x g blocks of X zero-padded to multiples of g (row-major block
    index), each of size ceil(rows/g) x ceil(cols/g)."""
    r, c = X.shape
    hr, hc = -(-r // g), -(-c // g)
    P = np.zeros((g * hr, g * hc), dtype=X.dtype)
    P[:r, :c] = X
    return [P[a * hr:(a + 1) * hr, b * hc:(b + 1) * hc] for a in range(g) for b in range(g)], hr, hc


def bilinear(A, B, s: Scheme, C0=None):
    """C0 + A B through one level of scheme s (eq. bilinear): the blocks of
    A and B (zero-padded to multiples of g, exact over a ring), the operand
    sums S_r and T_r in ascending block order, the R products P_r = S_r T_r
    by the library matmul, and C_c = sum_r gamma[c, r] P_r in ascending r.
    int64 for integer input (exact over Z), float64 otherwise."""
    A = np.asarray(A)
    B = np.asarray(B)
    integer = A.dtype.kind in "iu" and B.dtype.kind in "iu"
    dt = np.int64 if integer else np.float64
    A = A.astype(dt)
    B = B.astype(dt)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    g = s.g
    Ab, hm, hk = _blocks(A, g)
    Bb, _, hn = _blocks(B, g)
    Cb = [np.zeros((hm, hn), dtype=dt) for _ in range(g * g)]
    for r in range(s.products):
        S = np.zeros((hm, hk), dtype=dt)
        T = np.zeros((hk, hn), dtype=dt)
        for p in range(g * g):
            if s.alpha[r, p]:
                S += s.alpha[r, p] * Ab[p]
            if s.beta[r, p]:
                T += s.beta[r, p] * Bb[p]
        P = S @ T
        for c in range(g * g):
            if s.gamma[c, r]:
                Cb[c] += s.gamma[c, r] * P
    C = np.zeros((g * hm, g * hn), dtype=dt)
    for c in range(g * g):
        i, j = divmod(c, g)
        C[i * hm:(i + 1) * hm, j * hn:(j + 1) * hn] = Cb[c]
    out = C[:m, :n]
    if C0 is not None:
        out = out + np.asarray(C0, dtype=dt)
    return out
