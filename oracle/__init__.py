"""Oracle: plain CPU reference implementations of what the library computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The product library
(``paper_1911_05328_amd``) never imports it and shares no code with it.

Contents (each function cites the passage of Tang, "Improving the Space-Time
Efficiency of Processor-Oblivious Matrix Multiplication Algorithms", that it
follows):

* ``brute``        -- the semiring product by its definition (Sec. 1, eq. mm-dac).
* ``rec8``         -- 8-way recursion in CO2 order (Fig. mm-n2).
* ``rec8_split``   -- the same with k-halves sent to temporaries at chosen
                      depths and merged by madd (Fig. mm-n3 = CO3; lazy
                      allocation of Sec. sar-mm: the k-half-0 product works on
                      the parent's storage).
* ``strassen``     -- Strassen as printed in Sec. strassen, and
                      Strassen-Winograd; int64 or float64.
* ``fp64_ref``     -- classical float64 product (library matmul as the step).
* ``rel_fro``      -- relative Frobenius error; ``componentwise_err`` and
                      ``row_rel_err``: the componentwise and per-row errors
                      (not in the paper).
* ``split_bf16``   -- bf16 round-to-nearest-even hi/lo split (not in the paper).
* ``split3_product_f64`` / ``split3_fp16_product_f64`` -- the value of the
                      BF16x3 / FP16x3 product set (not in the paper).
* ``mlp_ref``      -- float64 MLP forward/backward (not in the paper).
* ``regret_ref``   -- exhaustive search over timed schedules and the regret
                      of a pick (not in the paper).
* ``bilinear_ref`` -- one level of a general bilinear scheme (the bilinear
                      circuit of the closing remarks of Sec. strassen, eq.
                      bilinear): scheme builders, the matrix-multiplication
                      tensor check, and the level itself.

The C part lives in ``oracle.c`` and is compiled with gcc into
``liboracle.so`` next to this file (``build()``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

PLUS_TIMES, MIN_PLUS, MAX_PLUS, MAX_MIN, OR_AND = 0, 1, 2, 3, 4
I32_MIN = -(1 << 31)  # zero of (max, min)
INF = 1 << 30  # saturating sentinel of the integer semirings

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (OpenMP for the plain loops)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        lib.or_brute_i64.argtypes = [ctypes.c_int, I, I, I, P, I, P, I, P, I]
        lib.or_brute_f64.argtypes = [I, I, I, P, I, P, I, P, I]
        lib.or_rec8_i64.argtypes = [ctypes.c_int, I, I, I, P, I, P, I, P, I, I, ctypes.c_uint32, P]
        lib.or_rec8_f64.argtypes = [I, I, I, P, I, P, I, P, I, I, ctypes.c_uint32, P]
        lib.or_strassen_f64.argtypes = [ctypes.c_int, ctypes.c_int, I, I, I, P, P, P]
        lib.or_strassen_i64.argtypes = [ctypes.c_int, ctypes.c_int, I, I, I, P, P, P]
        lib.or_split_bf16.argtypes = [I, P, P, P]
        lib.or_f32_to_bf16_rne.argtypes = [ctypes.c_uint32]
        lib.or_split_fp16.argtypes = [I, P, P, P]
        lib.or_f32_to_fp16_rne.argtypes = [ctypes.c_uint32]
        lib.or_f32_to_fp16_rne.restype = ctypes.c_uint16
        lib.or_fp16_to_f64.argtypes = [ctypes.c_uint16]
        lib.or_fp16_to_f64.restype = ctypes.c_double
        lib.or_f32_to_bf16_rne.restype = ctypes.c_uint16
        for f in ("or_brute_i64", "or_brute_f64", "or_rec8_i64", "or_rec8_f64",
                  "or_strassen_f64", "or_strassen_i64", "or_split_bf16"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    """Threads the oracle's parallel loops may use (for timing it)."""
    _load().or_set_threads(int(n))


def semiring_zero(sr: int) -> int:
    """Additive identity: +INF for (min,+), -INF for (max,+), the smallest
    int32 for (max, min), 0 for (+,x) and for Boolean (or, and)."""
    if sr == MIN_PLUS:
        return INF
    if sr == MAX_PLUS:
        return -INF
    if sr == MAX_MIN:
        return I32_MIN
    return 0


def brute(sr: int, A, B, C0=None):
    """O-1: C = C0 (+) A (x) B by the definition of the semiring product
    (Sec. 1: C = A (x) B on a closed semiring; eq. mm-dac).

    Integer semirings run in int64 with saturation at the sentinel INF=2^30
    ((min,+), (max,+)); (max, min) takes min for (x) and max for (+) with the
    smallest int32 as zero; Boolean (or, and) works on 0/1; (+,x) runs in
    int64 for integer input and float64 otherwise.
    """
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2
    floating = sr == PLUS_TIMES and (A.dtype.kind == "f" or B.dtype.kind == "f")
    if floating:
        C = _f64(np.zeros((m, n)) if C0 is None else C0).copy()
        _load().or_brute_f64(m, n, k, _ptr(_f64(A)), k, _ptr(_f64(B)), n, _ptr(C), n)
        return C
    C = _i64(np.full((m, n), semiring_zero(sr)) if C0 is None else C0).copy()
    Ai, Bi = _i64(A), _i64(B)
    _load().or_brute_i64(sr, m, n, k, _ptr(Ai), k, _ptr(Bi), n, _ptr(C), n)
    return C


def rec8(sr: int, A, B, C0=None, b: int = 32, split_mask: int = 0, stats: bool = False):
    """O-2/O-3: recursive 8-way product C (+)= A (x) B with base dimension b.

    ``split_mask`` bit d: at recursion depth d the k-half-1 sub-products go to
    a temporary of the current C block's size, merged into C by madd after
    both halves (Fig. mm-n3, CO3; Fig. wrapper-sar-mm with the k-half-0
    product keeping the parent's storage).  split_mask=0 is CO2 (Fig. mm-n2).

    With ``stats`` also returns (temp_total, temp_peak, leaves): the summed
    size of every temporary requested, the peak live temporary size in a
    depth-first run, and the number of base-case products.
    """
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    _, n = B.shape
    st = np.zeros(3, dtype=np.int64)
    floating = sr == PLUS_TIMES and (A.dtype.kind == "f" or B.dtype.kind == "f")
    if floating:
        C = _f64(np.zeros((m, n)) if C0 is None else C0).copy()
        _load().or_rec8_f64(m, n, k, _ptr(_f64(A)), k, _ptr(_f64(B)), n, _ptr(C), n,
                            b, split_mask, _ptr(st))
    else:
        C = _i64(np.full((m, n), semiring_zero(sr)) if C0 is None else C0).copy()
        _load().or_rec8_i64(sr, m, n, k, _ptr(_i64(A)), k, _ptr(_i64(B)), n, _ptr(C), n,
                            b, split_mask, _ptr(st))
    if stats:
        return C, tuple(int(x) for x in st)
    return C


def rec8_split(sr: int, A, B, C0=None, b: int = 32, split_levels: int = 0,
               first_split_depth: int = 0, stats: bool = False):
    """O-3 with the split depths given as a contiguous range: temporaries at
    depths [first_split_depth, first_split_depth + split_levels).

    first_split_depth=0 is CO3 restricted to the top levels; a positive
    first_split_depth is the STAR hybrid (Sec. star-mm): no temporaries above
    the switching depth, temporaries below it.
    """
    mask = 0
    for d in range(first_split_depth, first_split_depth + split_levels):
        mask |= 1 << d
    return rec8(sr, A, B, C0, b=b, split_mask=mask, stats=stats)


def rec_rect(sr: int, A, B, C0=None, b: int = 8, stats: bool = False):
    """The recursion for rectangular products: while max(m, n, k) > b, halve
    the largest of m, n, k (ceil half first; rows, then columns, then k on
    ties) -- k halves one after the other into the same C block, as CO2 does
    -- and at the leaves take the product by its definition (O-1).  Integer
    semirings in int64 (saturating as in brute); (+,x) float input in
    float64.  With ``stats`` also returns the number of leaves."""
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    _, n = B.shape
    floating = sr == PLUS_TIMES and (A.dtype.kind == "f" or B.dtype.kind == "f")
    if floating:
        C = _f64(np.zeros((m, n)) if C0 is None else C0).copy()
    else:
        C = _i64(np.full((m, n), semiring_zero(sr)) if C0 is None else C0).copy()
    leaves = [0]

    def rec(r0, r1, c0, c1, k0, k1):
        mm, nn, kk = r1 - r0, c1 - c0, k1 - k0
        if mm == 0 or nn == 0 or kk == 0:
            return
        if max(mm, nn, kk) <= b:
            C[r0:r1, c0:c1] = brute(sr, A[r0:r1, k0:k1], B[k0:k1, c0:c1], C[r0:r1, c0:c1])
            leaves[0] += 1
        elif mm >= nn and mm >= kk:
            h = r0 + (mm + 1) // 2
            rec(r0, h, c0, c1, k0, k1)
            rec(h, r1, c0, c1, k0, k1)
        elif nn >= kk:
            h = c0 + (nn + 1) // 2
            rec(r0, r1, c0, h, k0, k1)
            rec(r0, r1, h, c1, k0, k1)
        else:
            h = k0 + (kk + 1) // 2
            rec(r0, r1, c0, c1, k0, h)
            rec(r0, r1, c0, c1, h, k1)

    rec(0, m, 0, n, 0, k)
    return (C, leaves[0]) if stats else C


STRASSEN_CLASSIC, STRASSEN_WINOGRAD = 0, 1


def strassen(A, B, depth: int, variant: int = STRASSEN_WINOGRAD):
    """O-4: P = A B through ``depth`` levels of Strassen (variant 0: the seven
    products as printed in Sec. strassen) or Strassen-Winograd (variant 1),
    then the classical product.  Integer input runs in int64 (exact over Z),
    float input in float64.  Odd dimensions are padded with zeros per level.
    """
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    _, n = B.shape
    if A.dtype.kind in "iu" and B.dtype.kind in "iu":
        P = np.zeros((m, n), dtype=np.int64)
        _load().or_strassen_i64(variant, depth, m, n, k, _ptr(_i64(A)), _ptr(_i64(B)), _ptr(P))
    else:
        P = np.zeros((m, n), dtype=np.float64)
        _load().or_strassen_f64(variant, depth, m, n, k, _ptr(_f64(A)), _ptr(_f64(B)), _ptr(P))
    return P


def star_strassen(A, B, top: int, depth: int, variant: int = STRASSEN_WINOGRAD, C0=None):
    """STAR-Strassen (Thm. star-strassen-1): ``top`` levels of the 8-way
    recursion (TAR-MM: each C quadrant receives its two k-half products,
    k-half 0 first), then ``depth`` Strassen levels (O-4) on each of the 8^top
    sub-products.  Halves are ceil / floor as everywhere else.  int64 for
    integer input, float64 otherwise."""
    A = np.asarray(A)
    B = np.asarray(B)
    m, k = A.shape
    _, n = B.shape
    integer = A.dtype.kind in "iu" and B.dtype.kind in "iu"
    dt = np.int64 if integer else np.float64
    C = np.zeros((m, n), dtype=dt) if C0 is None else np.array(C0, dtype=dt)

    def rec(r0, r1, c0, c1, k0, k1, level):
        if r1 <= r0 or c1 <= c0 or k1 <= k0:
            return
        if level == top:
            C[r0:r1, c0:c1] += strassen(A[r0:r1, k0:k1], B[k0:k1, c0:c1], depth, variant).astype(dt)
            return
        rh, ch, kh = r0 + (r1 - r0 + 1) // 2, c0 + (c1 - c0 + 1) // 2, k0 + (k1 - k0 + 1) // 2
        for (ra, rb) in ((r0, rh), (rh, r1)):
            for (ca, cb) in ((c0, ch), (ch, c1)):
                rec(ra, rb, ca, cb, k0, kh, level + 1)
                rec(ra, rb, ca, cb, kh, k1, level + 1)

    rec(0, m, 0, n, 0, k, 0)
    return C


def fp64_ref(A, B, C0=None):
    """O-5: classical product in float64 of the given (fp32/bf16-valued) inputs.
    The library matmul is the step; accumulation is float64."""
    R = np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)
    if C0 is not None:
        R = R + np.asarray(C0, dtype=np.float64)
    return R


def fp64_rows(A, B, rows, C0=None):
    """float64 reference for selected output rows only (sampled parity at full size)."""
    rows = np.asarray(rows)
    R = np.asarray(A, dtype=np.float64)[rows] @ np.asarray(B, dtype=np.float64)
    if C0 is not None:
        R = R + np.asarray(C0, dtype=np.float64)[rows]
    return R


def rel_fro(C, R) -> float:
    """O-6: ||C - R||_F / ||R||_F in float64."""
    C = np.asarray(C, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    den = np.linalg.norm(R)
    return float(np.linalg.norm(C - R) / (den if den > 0 else 1.0))


def componentwise_err(C, R, A, B) -> float:
    """O-6: max over (i, j) of |C - R|_ij / (|A| |B|)_ij in float64 -- the error
    measured against the bound a classical product's rounding scales with.
    Entries with (|A| |B|)_ij = 0 have R_ij = 0 and count only if C_ij != 0
    (then the error is infinite)."""
    C = np.asarray(C, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    M = np.abs(np.asarray(A, dtype=np.float64)) @ np.abs(np.asarray(B, dtype=np.float64))
    D = np.abs(C - R)
    zero = M == 0
    if np.any(D[zero] != 0):
        return float("inf")
    return float(np.max(D[~zero] / M[~zero])) if np.any(~zero) else 0.0


def row_rel_err(C, R) -> np.ndarray:
    """O-6: per-row relative error ||C_i - R_i|| / ||R_i|| (float64), the
    figure that shows small rows next to large ones; a zero row of R gives
    the absolute error of that row."""
    C = np.asarray(C, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    num = np.linalg.norm(C - R, axis=1)
    den = np.linalg.norm(R, axis=1)
    return num / np.where(den > 0, den, 1.0)


def split_bf16(x):
    """O-7: hi = bf16_rne(x), lo = bf16_rne(x - hi); returns (hi, lo) as uint16 bit
    patterns.  Rounding written from the bit-level definition of round to
    nearest, ties to even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty(x.shape, dtype=np.uint16)
    lo = np.empty(x.shape, dtype=np.uint16)
    _load().or_split_bf16(x.size, _ptr(x), _ptr(hi), _ptr(lo))
    return hi, lo


def split_fp16(x):
    """O-7 (FP16): hi = fp16_rne(x), lo = fp16_rne(x - hi) as uint16 bit
    patterns; rounding written from the bit-level definition of binary16
    round to nearest, ties to even (normals, subnormals, overflow)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty(x.shape, dtype=np.uint16)
    lo = np.empty(x.shape, dtype=np.uint16)
    _load().or_split_fp16(x.size, _ptr(x), _ptr(hi), _ptr(lo))
    return hi, lo


def f32_to_fp16_bits(x) -> np.ndarray:
    """fp16_rne of each float32 value (uint16 bit patterns), one value at a time."""
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    f = _load().or_f32_to_fp16_rne
    return np.array([f(int(b)) for b in x.view(np.uint32)], dtype=np.uint16)


def fp16_bits_to_f64(u16) -> np.ndarray:
    """Value of binary16 bit patterns, in float64 (decoded by the oracle)."""
    f = _load().or_fp16_to_f64
    u = np.asarray(u16, dtype=np.uint16)
    return np.array([f(int(b)) for b in u.ravel()], dtype=np.float64).reshape(u.shape)


def pow2_scales(absmax, growth):
    """Power-of-two scale per row (or column): 2^(13 - ilogb(growth * absmax)),
    so that growth * absmax * scale < 2^14 (fp16 normal range with headroom);
    1 where absmax is 0.  `growth` bounds how much the Strassen pre-additions
    can enlarge an entry (2^d classic, 4^d Winograd, 1 without Strassen)."""
    b = np.asarray(absmax, dtype=np.float64) * growth
    e = np.where(b > 0, 13 - np.floor(np.log2(np.where(b > 0, b, 1.0))), 0.0)
    return np.ldexp(1.0, e.astype(np.int64))


def split3_fp16_product_f64(A, B):
    """FP16x3 with exact per-row (A) / per-column (B) power-of-two scaling,
    before fp32 rounding: scale, split into fp16 hi/lo, Ah Bh + Ah Bl + Al Bh
    in float64, unscale.  Diagnostic for the split error."""
    A = np.asarray(A, dtype=np.float32)
    B = np.asarray(B, dtype=np.float32)
    sa = pow2_scales(np.abs(A).max(axis=1), 1.0)
    sb = pow2_scales(np.abs(B).max(axis=0), 1.0)
    As = (A.astype(np.float64) * sa[:, None]).astype(np.float32)
    Bs = (B.astype(np.float64) * sb[None, :]).astype(np.float32)
    ah, al = split_fp16(As)
    bh, bl = split_fp16(Bs)
    Ah, Al = (np.asarray(ah).view(np.float16).astype(np.float64), np.asarray(al).view(np.float16).astype(np.float64))
    Bh, Bl = (np.asarray(bh).view(np.float16).astype(np.float64), np.asarray(bl).view(np.float16).astype(np.float64))
    return (Ah @ Bh + Ah @ Bl + Al @ Bh) / (sa[:, None] * sb[None, :])


def bf16_bits_to_f64(u16) -> np.ndarray:
    """Value of bf16 bit patterns, in float64."""
    u = np.asarray(u16, dtype=np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def split3_product_f64(A, B):
    """Value that an exact split-precision product computes before fp32
    rounding: Ah Bh + Ah Bl + Al Bh with the bf16 split above (the lo*lo term
    is dropped), accumulated in float64.  Diagnostic for the split error."""
    ah, al = split_bf16(A)
    bh, bl = split_bf16(B)
    Ah, Al = bf16_bits_to_f64(ah), bf16_bits_to_f64(al)
    Bh, Bl = bf16_bits_to_f64(bh), bf16_bits_to_f64(bl)
    return Ah @ Bh + Ah @ Bl + Al @ Bh


# ---- Strassen's space-bounded layouts (Lemma par-strassen, Lemma
# sar-strassen, Thm. star-strassen-2) ------------------------------------
#
# One Strassen level, in the printed form (variant 0) or Strassen-Winograd
# (variant 1), as the quadrant combinations each product takes and each C
# quadrant receives.  Written out here from the formulas, independent of the
# C implementation above; quadrants are indexed q = 2 i + j.
_SW_CLASSIC = (
    # (A combination, B combination, C quadrants with their signs)
    ({0: 1, 3: 1}, {0: 1, 3: 1}, {0: 1, 3: 1}),    # P1 = (A00 + A11)(B00 + B11)
    ({2: 1, 3: 1}, {0: 1}, {2: 1, 3: -1}),         # P2 = (A10 + A11) B00
    ({0: 1}, {1: 1, 3: -1}, {1: 1, 3: 1}),         # P3 = A00 (B01 - B11)
    ({3: 1}, {2: 1, 0: -1}, {0: 1, 2: 1}),         # P4 = A11 (B10 - B00)
    ({0: 1, 1: 1}, {3: 1}, {0: -1, 1: 1}),         # P5 = (A00 + A01) B11
    ({2: 1, 0: -1}, {0: 1, 1: 1}, {3: 1}),         # P6 = (A10 - A00)(B00 + B01)
    ({1: 1, 3: -1}, {2: 1, 3: 1}, {0: 1}),         # P7 = (A01 - A11)(B10 + B11)
)
# Strassen-Winograd with S1 = A10 + A11, S2 = S1 - A00, S3 = A00 - A10,
# S4 = A01 - S2, T1 = B01 - B00, T2 = B11 - T1, T3 = B11 - B01,
# T4 = T2 - B10, products M1 = A00 B00, M2 = A01 B10, M3 = S4 B11,
# M4 = A11 T4, M5 = S1 T1, M6 = S2 T2, M7 = S3 T3, and C00 = M1 + M2,
# U2 = M1 + M6 + M7 (C10 = U2 - M4, C11 = U2 + M5), C01 = M1 + M6 + M5 + M3,
# each sum expanded over quadrants.
_SW_WINOGRAD = (
    ({0: 1}, {0: 1}, {0: 1, 1: 1, 2: 1, 3: 1}),
    ({1: 1}, {2: 1}, {0: 1}),
    ({0: 1, 1: 1, 2: -1, 3: -1}, {3: 1}, {1: 1}),
    ({3: 1}, {0: 1, 1: -1, 2: -1, 3: 1}, {2: -1}),
    ({2: 1, 3: 1}, {1: 1, 0: -1}, {1: 1, 3: 1}),
    ({2: 1, 3: 1, 0: -1}, {0: 1, 1: -1, 3: 1}, {1: 1, 2: 1, 3: 1}),
    ({0: 1, 2: -1}, {3: 1, 1: -1}, {2: 1, 3: 1}),
)


def _quadrants(X):
    """The four quadrants of X after zero-padding each dimension to even."""
    r, c = X.shape
    hr, hc = (r + 1) // 2, (c + 1) // 2
    P = np.zeros((2 * hr, 2 * hc), dtype=X.dtype)
    P[:r, :c] = X
    return [P[:hr, :hc], P[:hr, hc:], P[hr:, :hc], P[hr:, hc:]]


def _combine(quads, coefs):
    out = np.zeros_like(quads[0])
    for q, c in sorted(coefs.items()):
        out += c * quads[q]
    return out


def strassen_layout(A, B, depth: int, variant: int = STRASSEN_CLASSIC, layout: int = 0, C0=None):
    """C0 + A B through ``depth`` Strassen levels whose order of evaluation
    and temporary storage follow ``layout``: bit l (l = 0 the top level) set
    makes level l depth-first, as SAR-Strassen does (Lemma sar-strassen: the
    seven products one after another, each with its operands S_r, T_r formed
    on the fly and its product P_r, three temporaries of the level's size
    reused by the next product, P_r added into the quadrants of C at once);
    clear makes it breadth-first, as the straightforward parallel Strassen
    does (Lemma par-strassen: every S_r, T_r that is not a bare quadrant and
    all seven P_r exist at once, 17 quadrant-size temporaries for the printed
    variant, and all seven sub-products run concurrently).  Breadth-first
    levels above depth-first ones are Thm. star-strassen-2.

    Returns (C, peak) where peak counts the temporary elements live at once
    when every breadth-first level's seven sub-products run concurrently and
    every depth-first level's run in turn: the space recurrences
    S(n) = 7 S(n/2) + t (n/2)^2 (breadth-first, t temporaries) and
    S(n) = S(n/2) + 3 (n/2)^2 (depth-first).  Values: int64 for integer
    input (exact over Z), float64 otherwise; odd dimensions zero-padded per
    level."""
    A = np.asarray(A)
    B = np.asarray(B)
    integer = A.dtype.kind in "iu" and B.dtype.kind in "iu"
    dt = np.int64 if integer else np.float64
    table = _SW_CLASSIC if variant == STRASSEN_CLASSIC else _SW_WINOGRAD

    def rec(X, Y, level):
        """(product X Y, peak temporaries of computing it)"""
        if level == depth:
            return X @ Y, 0
        xq, yq = _quadrants(X), _quadrants(Y)
        hr, hk = xq[0].shape
        hc = yq[0].shape[1]
        out = [np.zeros((hr, hc), dtype=dt) for _ in range(4)]
        if (layout >> level) & 1:
            # depth-first: S_r, T_r, P_r one product at a time, space reused
            child_peak = 0
            for sa, sb, sc in table:
                S = _combine(xq, sa)
                T = _combine(yq, sb)
                P, cp = rec(S, T, level + 1)
                child_peak = max(child_peak, cp)
                for q, c in sc.items():
                    out[q] += c * P
            peak = hr * hk + hk * hc + hr * hc + child_peak
        else:
            # breadth-first: all operands first, then all seven products
            S = [_combine(xq, sa) for sa, _, _ in table]
            T = [_combine(yq, sb) for _, sb, _ in table]
            temps = sum(hr * hk for sa, _, _ in table if len(sa) > 1) + \
                sum(hk * hc for _, sb, _ in table if len(sb) > 1) + 7 * hr * hc
            results = [rec(S[r], T[r], level + 1) for r in range(7)]
            for r, (_, _, sc) in enumerate(table):
                for q, c in sc.items():
                    out[q] += c * results[r][0]
            peak = temps + sum(cp for _, cp in results)
        full = np.block([[out[0], out[1]], [out[2], out[3]]])
        return full[:X.shape[0], :Y.shape[1]], peak

    P, peak = rec(A.astype(dt), B.astype(dt), 0)
    C = P if C0 is None else np.asarray(C0, dtype=dt) + P
    return C, peak
