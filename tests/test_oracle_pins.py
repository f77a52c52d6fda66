"""Pins the oracle to facts other than itself: library routines, closed forms,
algebraic identities and brute force on tiny inputs.  CPU only.

A plausible mistake in the oracle (a dropped term, a wrong sign or index, a
transposed operand, a missed saturation) fails at least one of these.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
INF = oracle.INF


def setup_module(_):
    oracle.build(force=False)


# ---------------------------------------------------------------- O-1 brute


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (5, 7, 3), (33, 17, 65), (64, 64, 64)])
def test_brute_plus_times_int64_equals_numpy(m, n, k):
    g = np.random.default_rng(m * 1000 + n * 10 + k)
    A = g.integers(-1000, 1000, (m, k))
    B = g.integers(-1000, 1000, (k, n))
    C0 = g.integers(-1000, 1000, (m, n))
    assert np.array_equal(oracle.brute(oracle.PLUS_TIMES, A, B, C0), C0 + A @ B)


def test_brute_plus_times_f64_integer_valued_exact():
    g = np.random.default_rng(5)
    A = g.integers(-8, 9, (40, 50)).astype(np.float64)
    B = g.integers(-8, 9, (50, 30)).astype(np.float64)
    assert np.array_equal(oracle.brute(oracle.PLUS_TIMES, A, B), A @ B)


def _identity(sr, n):
    one = {oracle.MAX_MIN: (1 << 31) - 1, oracle.OR_AND: 1}.get(sr, 0)
    zero = oracle.semiring_zero(sr)
    I = np.full((n, n), zero, dtype=np.int64)
    np.fill_diagonal(I, one)
    return I


@pytest.mark.parametrize("sr", [oracle.MIN_PLUS, oracle.MAX_PLUS, oracle.MAX_MIN, oracle.OR_AND])
def test_brute_semiring_identity(sr):
    n = 23
    A = si.semiring_operand(sr, 1, (n, n)).astype(np.int64)
    I = _identity(sr, n)
    assert np.array_equal(oracle.brute(sr, I, A), A)
    assert np.array_equal(oracle.brute(sr, A, I), A)


@pytest.mark.parametrize("sr", [oracle.MIN_PLUS, oracle.MAX_PLUS, oracle.MAX_MIN, oracle.OR_AND])
def test_brute_zero_row_annihilates(sr):
    # An all-zero (i.e. all-INF) row of A gives an all-zero row of C: zero
    # annihilates under (x) and is neutral under (+).
    n = 19
    A = si.semiring_operand(sr, 3, (n, n)).astype(np.int64)
    B = si.semiring_operand(sr, 4, (n, n)).astype(np.int64)
    A[5, :] = oracle.semiring_zero(sr)
    C = oracle.brute(sr, A, B)
    assert (C[5] == oracle.semiring_zero(sr)).all()


def test_minplus_path_graph_closed_form():
    # Path 0-1-...-n-1, unit weights, 0 on the diagonal.  (A (x) A)_ij = |i-j|
    # for |i-j| <= 2 else INF; ceil(log2 n) squarings give |i-j| everywhere.
    n = 37
    A = np.full((n, n), INF, dtype=np.int64)
    for i in range(n):
        A[i, i] = 0
        if i + 1 < n:
            A[i, i + 1] = A[i + 1, i] = 1
    d = np.abs(np.arange(n)[:, None] - np.arange(n)[None, :])
    A2 = oracle.brute(oracle.MIN_PLUS, A, A)
    assert np.array_equal(A2, np.where(d <= 2, d, INF))
    D = A
    for _ in range(math.ceil(math.log2(n))):
        D = oracle.brute(oracle.MIN_PLUS, D, D)
    assert np.array_equal(D, d)


def test_minplus_squaring_matches_scipy_shortest_paths():
    scipy_csgraph = pytest.importorskip("scipy.sparse.csgraph")
    n = 48
    g = np.random.default_rng(11)
    W = g.integers(1, 50, (n, n)).astype(np.int64)
    W[g.random((n, n)) < 0.85] = INF
    np.fill_diagonal(W, 0)
    dense = np.where(W >= INF, 0, W).astype(np.float64)  # 0 = no edge for csgraph
    ref = scipy_csgraph.shortest_path(dense, method="FW", directed=True)
    D = W
    for _ in range(math.ceil(math.log2(n))):
        D = oracle.brute(oracle.MIN_PLUS, D, D)
    expect = np.where(np.isinf(ref), INF, ref).astype(np.int64)
    assert np.array_equal(D, expect)


def test_maxplus_is_negated_minplus():
    # max(a+b) = -min((-a)+(-b)); the sentinels map INF <-> -INF.
    g = 29
    A = si.maxplus_i32(7, (g, 31)).astype(np.int64)
    B = si.maxplus_i32(8, (31, 13)).astype(np.int64)
    C_max = oracle.brute(oracle.MAX_PLUS, A, B)
    C_min = oracle.brute(oracle.MIN_PLUS, -A, -B)
    assert np.array_equal(C_max, -C_min)


def test_minplus_saturates_inf_plus_inf():
    A = np.array([[INF, 5]], dtype=np.int64)
    B = np.array([[INF], [INF]], dtype=np.int64)
    assert oracle.brute(oracle.MIN_PLUS, A, B)[0, 0] == INF
    A = np.array([[INF - 3]], dtype=np.int64)
    B = np.array([[10]], dtype=np.int64)
    assert oracle.brute(oracle.MIN_PLUS, A, B)[0, 0] == INF


def test_minplus_negative_directed_path_closed_form():
    # Directed path i -> i+1 of weight -1, 0 on the diagonal.  After t
    # squarings, D_ij = -(j - i) for 0 <= j - i <= 2^t, INF otherwise (an INF
    # entry times a negative one must stay INF).
    n = 41
    A = np.full((n, n), INF, dtype=np.int64)
    for i in range(n):
        A[i, i] = 0
        if i + 1 < n:
            A[i, i + 1] = -1
    d = np.arange(n)[None, :] - np.arange(n)[:, None]  # j - i
    D = A
    for t in range(1, math.ceil(math.log2(n)) + 1):
        D = oracle.brute(oracle.MIN_PLUS, D, D)
        assert np.array_equal(D, np.where((d >= 0) & (d <= 2 ** t), -d, INF)), t


def test_minplus_negative_dag_matches_bellman_ford():
    # Shortest paths with negative edge weights (a DAG, so no negative
    # cycles): (min,+) squaring against scipy's Bellman-Ford.
    scipy_csgraph = pytest.importorskip("scipy.sparse.csgraph")
    n = 45
    g = np.random.default_rng(12)
    W = g.integers(-40, 61, (n, n)).astype(np.int64)
    W[W == 0] = 1  # csgraph reads 0 as "no edge"
    W[(g.random((n, n)) < 0.8) | (np.arange(n)[:, None] >= np.arange(n)[None, :])] = INF
    np.fill_diagonal(W, 0)
    dense = np.where(W >= INF, 0, W).astype(np.float64)
    ref = scipy_csgraph.shortest_path(dense, method="BF", directed=True)
    D = W
    for _ in range(math.ceil(math.log2(n))):
        D = oracle.brute(oracle.MIN_PLUS, D, D)
    assert (ref[np.isfinite(ref)] < 0).any()
    assert np.array_equal(D, np.where(np.isinf(ref), INF, ref).astype(np.int64))


def test_maxplus_longest_dag_paths_are_negated_shortest():
    # (max,+) squaring gives longest paths: the negated Bellman-Ford distances
    # of the negated weights.
    scipy_csgraph = pytest.importorskip("scipy.sparse.csgraph")
    n = 39
    g = np.random.default_rng(13)
    W = g.integers(-50, 51, (n, n)).astype(np.int64)
    W[W == 0] = 2
    W[(g.random((n, n)) < 0.75) | (np.arange(n)[:, None] >= np.arange(n)[None, :])] = -INF
    np.fill_diagonal(W, 0)
    dense = np.where(W <= -INF, 0, -W).astype(np.float64)
    ref = -scipy_csgraph.shortest_path(dense, method="BF", directed=True)
    D = W
    for _ in range(math.ceil(math.log2(n))):
        D = oracle.brute(oracle.MAX_PLUS, D, D)
    assert (ref[np.isfinite(ref)] > 0).any()
    assert np.array_equal(D, np.where(np.isinf(ref), -INF, ref).astype(np.int64))


def test_wide_domain_extremes():
    # The checked domain's corner cases: INF with a negative partner stays
    # INF, the most negative sum -2^31 is kept, a sum reaching INF saturates.
    A = np.array([[INF, -INF, INF - 1, -5]], dtype=np.int64)
    B = np.array([[-7], [-INF], [3], [INF]], dtype=np.int64)
    C = oracle.brute(oracle.MIN_PLUS, A, B)
    assert C[0, 0] == -2 ** 31
    terms = [oracle.brute(oracle.MIN_PLUS, A[:, [l]], B[[l], :])[0, 0] for l in range(4)]
    assert terms == [INF, -2 ** 31, INF, INF]
    # (max,+): -INF with a positive partner stays -INF; the largest sum 2^31 - 2
    A = np.array([[-INF, INF - 1, 5]], dtype=np.int64)
    B = np.array([[INF - 1], [INF - 1], [-INF]], dtype=np.int64)
    terms = [oracle.brute(oracle.MAX_PLUS, A[:, [l]], B[[l], :])[0, 0] for l in range(3)]
    assert terms == [-INF, 2 ** 31 - 2, -INF]


def test_wide_generator_domain():
    for sr, lo, hi, sentinel in ((1, -INF, INF, INF), (2, -INF + 1, INF - 1, -INF)):
        x = si.wide_i32(sr, 5, (300, 300)).astype(np.int64)
        finite = x[x != sentinel]
        assert finite.min() >= lo and finite.max() <= hi
        assert (finite < -(1 << 28)).any() and (finite > (1 << 28)).any() and (x == sentinel).any()


def test_minplus_numpy_broadcast_small():
    # Independent small-n evaluation: saturated pairwise sums reduced by min.
    g = np.random.default_rng(2)
    A = si.minplus_i32(21, (17, 23)).astype(np.int64)
    B = si.minplus_i32(22, (23, 9)).astype(np.int64)
    s = A[:, :, None] + B[None, :, :]
    s = np.where((A[:, :, None] >= INF) | (B[None, :, :] >= INF), INF, np.minimum(s, INF))
    C0 = np.where(g.random((17, 9)) < 0.5, INF, g.integers(0, 1 << 20, (17, 9)))
    assert np.array_equal(oracle.brute(oracle.MIN_PLUS, A, B, C0), np.minimum(C0, s.min(axis=1)))


def test_boolean_equals_numpy_integer_product():
    # Boolean (or, and): C_ij is true iff C0_ij or some A_il and B_lj are;
    # the integer product A B counts those l (numpy matmul, int64).
    for (m, n, k, d) in [(1, 1, 1, 0.5), (17, 23, 31, 0.1), (64, 48, 200, 0.02), (40, 40, 40, 0.0)]:
        A = si.bool_i32(m + k, (m, k), d).astype(np.int64)
        B = si.bool_i32(n + k, (k, n), d).astype(np.int64)
        C0 = si.bool_i32(m + n, (m, n), 0.05).astype(np.int64)
        expect = ((A @ B) > 0) | (C0 > 0)
        assert np.array_equal(oracle.brute(oracle.OR_AND, A, B, C0), expect.astype(np.int64))


def test_boolean_squaring_is_reachability():
    # (I or G) squared ceil(log2 n) times is the reachability relation,
    # against scipy's breadth-first shortest paths (finite = reachable).
    scipy_csgraph = pytest.importorskip("scipy.sparse.csgraph")
    n = 60
    G = si.bool_i32(77, (n, n), 0.03).astype(np.int64)
    R = G.copy()
    np.fill_diagonal(R, 1)
    for _ in range(math.ceil(math.log2(n))):
        R = oracle.brute(oracle.OR_AND, R, R)
    d = scipy_csgraph.shortest_path(G.astype(np.float64), method="D", directed=True, unweighted=True)
    assert np.array_equal(R, np.isfinite(d).astype(np.int64))


def test_maxmin_threshold_decomposition():
    # (max, min): C_ij >= t iff C0_ij >= t or some l has A_il >= t and
    # B_lj >= t, for every threshold t -- a Boolean product per threshold,
    # evaluated by numpy's integer matmul.  Together over all t this fixes C.
    g = np.random.default_rng(31)
    m, n, k = 19, 27, 35
    A = si.maxmin_i32(41, (m, k)).astype(np.int64)
    B = si.maxmin_i32(42, (k, n)).astype(np.int64)
    C0 = si.maxmin_i32(43, (m, n), 0.7).astype(np.int64)
    C = oracle.brute(oracle.MAX_MIN, A, B, C0)
    vals = np.unique(np.concatenate([A.ravel(), B.ravel(), C0.ravel()]))
    for t in np.concatenate([g.choice(vals, 200), [vals[0], vals[-1]]]):
        hit = ((A >= t).astype(np.int64) @ (B >= t).astype(np.int64)) > 0
        assert np.array_equal(C >= t, hit | (C0 >= t)), t


def test_maxmin_squaring_is_widest_path():
    # Widest (bottleneck) paths of an undirected graph: the capacity between
    # i and j is the smallest edge on their path in a maximum spanning tree
    # (scipy's minimum spanning tree of the negated capacities).
    scipy_csgraph = pytest.importorskip("scipy.sparse.csgraph")
    n = 40
    g = np.random.default_rng(12)
    cap = g.integers(1, 1000, (n, n))
    cap = np.triu(cap, 1)
    cap[np.triu(g.random((n, n)) < 0.8, 1)] = 0  # sparse; may be disconnected
    cap = cap + cap.T
    W = np.where(cap > 0, cap, si.I32_MIN).astype(np.int64)
    np.fill_diagonal(W, si.I32_MAX)
    D = W
    for _ in range(math.ceil(math.log2(n))):
        D = oracle.brute(oracle.MAX_MIN, D, D)
    T = scipy_csgraph.minimum_spanning_tree(-cap.astype(np.float64)).toarray()
    T = -(T + T.T)  # tree edges with their capacities, 0 = none
    expect = np.full((n, n), si.I32_MIN, dtype=np.int64)
    for s in range(n):  # walk the tree from s, carrying the smallest edge so far
        expect[s, s] = si.I32_MAX
        stack = [s]
        while stack:
            u = stack.pop()
            for v in np.nonzero(T[u])[0]:
                if expect[s, v] == si.I32_MIN and v != s:
                    expect[s, v] = min(expect[s, u], int(T[u, v]))
                    stack.append(v)
    assert np.array_equal(D, expect)


# ---------------------------------------------------------- O-2 / O-3 recursion

SIZES = [1, 2, 3, 5, 8, 17, 31, 32, 33]


@pytest.mark.parametrize("sr", [oracle.MIN_PLUS, oracle.MAX_PLUS, oracle.MAX_MIN, oracle.OR_AND, oracle.PLUS_TIMES])
def test_rec8_equals_brute_all_plans(sr):
    g = np.random.default_rng(sr + 100)
    for m, n, k in itertools.product(SIZES, SIZES[::3], SIZES[::2]):
        if sr == oracle.PLUS_TIMES:
            A = g.integers(-50, 50, (m, k))
            B = g.integers(-50, 50, (k, n))
            C0 = g.integers(-50, 50, (m, n))
        else:
            A = si.semiring_operand(sr, m * 7 + k, (m, k)).astype(np.int64)
            B = si.semiring_operand(sr, n * 11 + k, (k, n)).astype(np.int64)
            C0 = si.semiring_operand(sr, m + n, (m, n)).astype(np.int64)
        ref = oracle.brute(sr, A, B, C0)
        for b in (1, 2, 4, 8):
            for mask in (0, 1, 3, 2, 0xFF):
                got = oracle.rec8(sr, A, B, C0, b=b, split_mask=mask)
                assert np.array_equal(got, ref), (m, n, k, b, mask)


@pytest.mark.parametrize("sr", [oracle.MIN_PLUS, oracle.MAX_MIN, oracle.OR_AND, oracle.PLUS_TIMES])
def test_rec_rect_equals_brute_and_leaf_counts(sr):
    # Halving the largest dimension computes the same product as the
    # definition, for thin, flat, deep and square shapes.
    g = np.random.default_rng(sr + 300)
    for (m, n, k) in [(1, 1, 1), (1, 40, 3), (37, 1, 5), (2, 3, 61), (33, 17, 9), (16, 16, 16), (5, 70, 70)]:
        if sr == oracle.PLUS_TIMES:
            A, B, C0 = g.integers(-50, 50, (m, k)), g.integers(-50, 50, (k, n)), g.integers(-50, 50, (m, n))
        else:
            A = si.semiring_operand(sr, m + k, (m, k)).astype(np.int64)
            B = si.semiring_operand(sr, n + k, (k, n)).astype(np.int64)
            C0 = si.semiring_operand(sr, m + n, (m, n)).astype(np.int64)
        ref = oracle.brute(sr, A, B, C0)
        for b in (1, 2, 4, 8):
            assert np.array_equal(oracle.rec_rect(sr, A, B, C0, b=b), ref), (m, n, k, b)
    # leaf counts: a power-of-two cube down to b = 1 has 8^L leaves (as the
    # 8-way recursion); a thin m x 1 x 1 product is m leaves; a 64 x 4 x 4
    # product with b = 4 halves m only: 16 leaves
    A = np.ones((8, 8), np.int64)
    assert oracle.rec_rect(oracle.PLUS_TIMES, A, A, b=1, stats=True)[1] == 8 ** 3
    assert oracle.rec_rect(oracle.PLUS_TIMES, np.ones((13, 1), np.int64), np.ones((1, 1), np.int64),
                           b=1, stats=True)[1] == 13
    assert oracle.rec_rect(oracle.PLUS_TIMES, np.ones((64, 4), np.int64), np.ones((4, 4), np.int64),
                           b=4, stats=True)[1] == 16


def test_rec8_f64_close_to_brute():
    g = np.random.default_rng(9)
    A = g.uniform(-1, 1, (65, 47))
    B = g.uniform(-1, 1, (47, 33))
    ref = A @ B
    for mask in (0, 1, 0xF):
        got = oracle.rec8(oracle.PLUS_TIMES, A, B, b=4, split_mask=mask)
        assert oracle.rel_fro(got, ref) < 1e-14


def test_co3_total_temporary_space_closed_form():
    # CO3 allocates n^3 - n^2 temporary elements in total (base case 1).
    for n, expect in GOLD["co3_total_temp"]["cases"]:
        assert expect == n ** 3 - n ** 2
        A = np.zeros((n, n), dtype=np.int64)
        _, (total, peak, leaves) = oracle.rec8(oracle.MIN_PLUS, A, A, b=1,
                                               split_mask=0xFFFF, stats=True)
        assert total == expect
        assert leaves == n ** 3
        # a depth-first run holds one temporary per level on the current path
        levels = int(math.log2(n))
        assert peak == sum((n >> d) ** 2 for d in range(levels))


def test_co2_requests_no_temporaries():
    # CO2 (no k-split anywhere) needs only the 3 n^2 of its inputs and output.
    assert GOLD["co2_io_space"]["value_in_n2"] == 3
    for n in (8, 16, 32):
        A = np.zeros((n, n), dtype=np.int64)
        C, (total, peak, leaves) = oracle.rec8(oracle.MIN_PLUS, A, A, b=1, split_mask=0, stats=True)
        assert total == 0 and peak == 0 and leaves == n ** 3
        assert A.size + A.size + C.size == GOLD["co2_io_space"]["value_in_n2"] * n * n


@pytest.mark.parametrize("j", [1, 2, 3])
def test_top_level_split_temp_closed_form(j):
    # Temporaries at the top j levels: (2^j - 1) n^2 elements.
    n = 64
    A = np.zeros((n, n), dtype=np.int64)
    _, (total, _, _) = oracle.rec8_split(oracle.MIN_PLUS, A, A, b=8, split_levels=j, stats=True)
    assert total == (2 ** j - 1) * n * n


def test_star_switch_depth_no_temps_above():
    # STAR hybrid: no temporaries above the switching depth k; below, the
    # same counts as CO3 restricted to depths >= k: sum_{d>=k} 8^d (n/2^d)^2.
    n, k = 32, 2
    A = np.zeros((n, n), dtype=np.int64)
    _, (total, _, _) = oracle.rec8_split(oracle.MIN_PLUS, A, A, b=1, split_levels=10,
                                         first_split_depth=k, stats=True)
    assert total == sum(8 ** d * (n >> d) ** 2 for d in range(k, 5))
    assert total == n * n * (n - 2 ** k)


# ----------------------------------------------------------------- O-4 Strassen


@pytest.mark.parametrize("variant", [oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD])
def test_strassen_seven_product_identity(variant):
    # Bilinearity: one Strassen level on 2x2 unit matrices E_ab, E_cd must
    # give delta_bc E_ad.  These 16 cases cover all 64 entries of the 2x2x2
    # matrix multiplication tensor.
    for a, b, c, d in itertools.product(range(2), repeat=4):
        X = np.zeros((2, 2), dtype=np.int64)
        Y = np.zeros((2, 2), dtype=np.int64)
        X[a, b] = 1
        Y[c, d] = 1
        P = oracle.strassen(X, Y, depth=1, variant=variant)
        E = np.zeros((2, 2), dtype=np.int64)
        if b == c:
            E[a, d] = 1
        assert np.array_equal(P, E), (variant, a, b, c, d)


@pytest.mark.parametrize("variant", [oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_int64_exact(variant, depth):
    g = np.random.default_rng(depth * 10 + variant)
    for m, n, k in [(128, 128, 128), (37, 53, 29), (64, 17, 100), (9, 9, 9)]:
        A = g.integers(-1024, 1025, (m, k))
        B = g.integers(-1024, 1025, (k, n))
        assert np.array_equal(oracle.strassen(A, B, depth, variant), A @ B)


@pytest.mark.parametrize("variant", [oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD])
def test_strassen_f64_error_bound(variant):
    g = np.random.default_rng(4)
    A = g.standard_normal((256, 256))
    B = g.standard_normal((256, 256))
    P = oracle.strassen(A, B, 3, variant)
    assert oracle.rel_fro(P, A @ B) < 1e-13


@pytest.mark.parametrize("top,depth", [(1, 1), (2, 1), (1, 2), (3, 0)])
def test_star_strassen_int64_exact_and_fp64_bound(top, depth):
    # 8-way levels above Strassen levels still compute the ring product:
    # exact over Z against numpy's int64 matmul, odd sizes included, and
    # within Strassen's float64 error bound on random reals.
    g = np.random.default_rng(top * 10 + depth)
    for (m, n, k) in [(37, 29, 51), (64, 64, 64), (1, 5, 3)]:
        A = g.integers(-1000, 1000, (m, k))
        B = g.integers(-1000, 1000, (k, n))
        C0 = g.integers(-1000, 1000, (m, n))
        for variant in (oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD):
            got = oracle.star_strassen(A, B, top, depth, variant, C0)
            assert np.array_equal(got, A.astype(np.int64) @ B.astype(np.int64) + C0), (m, n, k, variant)
    A = g.standard_normal((90, 70))
    B = g.standard_normal((70, 110))
    R = A @ B
    assert np.linalg.norm(oracle.star_strassen(A, B, top, depth) - R) / np.linalg.norm(R) < 1e-13


def test_strassen_wrong_sign_would_fail():
    # Sanity of the pin itself: flipping one post-addition sign in a numpy
    # re-derivation of the classic C11 changes the result.
    g = np.random.default_rng(1)
    A = g.integers(-5, 6, (2, 2))
    B = g.integers(-5, 6, (2, 2))
    P1 = (A[0, 0] + A[1, 1]) * (B[0, 0] + B[1, 1])
    P2 = (A[1, 0] + A[1, 1]) * B[0, 0]
    P3 = A[0, 0] * (B[0, 1] - B[1, 1])
    P6 = (A[1, 0] - A[0, 0]) * (B[0, 0] + B[0, 1])
    good = P1 + P3 - P2 + P6
    bad = P1 + P3 + P2 + P6
    assert good == (A @ B)[1, 1]
    assert bad != good or P2 == 0


# ---------------------------------------------------------------- O-5 / O-6


def test_fp64_ref_integer_exact_and_rows():
    A = si.small_int_f32(1, (70, 90))
    B = si.small_int_f32(2, (90, 50))
    R = oracle.fp64_ref(A, B)
    assert np.array_equal(R, oracle.brute(oracle.PLUS_TIMES, A.astype(np.int64), B.astype(np.int64)))
    rows = np.array([0, 13, 69])
    assert np.array_equal(oracle.fp64_rows(A, B, rows), R[rows])


def test_rel_fro_definition():
    R = np.array([[3.0, 4.0]])
    C = np.array([[3.0, 4.0 + 1e-3]])
    assert abs(oracle.rel_fro(C, R) - 1e-3 / 5.0) < 1e-15
    assert oracle.rel_fro(R, R) == 0.0


def test_componentwise_err_closed_forms():
    # nonnegative integer operands: |A||B| = A B = R, so perturbing one entry
    # of C by R_ij * 2^-10 gives exactly 2^-10
    rng = np.random.default_rng(5)
    A = rng.integers(1, 9, (6, 5)).astype(np.float64)
    B = rng.integers(1, 9, (5, 7)).astype(np.float64)
    R = A @ B
    C = R.copy()
    C[2, 3] += R[2, 3] * 2.0 ** -10
    assert oracle.componentwise_err(C, R, A, B) == 2.0 ** -10
    assert oracle.componentwise_err(R, R, A, B) == 0.0
    # cancellation: R = 1 - 1 = 0 but |A||B| = 2, so an error of 0.5 is 0.25
    # (a denominator of |R| or |A B| would make it infinite)
    A2 = np.array([[1.0, -1.0]])
    B2 = np.array([[1.0], [1.0]])
    assert oracle.componentwise_err(np.array([[0.5]]), A2 @ B2, A2, B2) == 0.25
    # a structurally zero entry (|A||B| = 0) counts only when C is nonzero there
    A3 = np.array([[0.0, 0.0], [1.0, 2.0]])
    B3 = np.eye(2)
    R3 = A3 @ B3
    assert oracle.componentwise_err(R3, R3, A3, B3) == 0.0
    C3 = R3.copy()
    C3[0, 1] = 1e-30
    assert oracle.componentwise_err(C3, R3, A3, B3) == float("inf")


def test_row_rel_err_shows_small_rows():
    # row 0 large, row 1 tiny: a 10% error on the tiny row hides in the
    # normwise figure (~2e-8) but is the per-row error of that row
    R = np.array([[3.0, 4.0], [0.0, 1e-6]])
    C = R + np.array([[0.0, 5e-3], [0.0, 1e-7]])
    e = oracle.row_rel_err(C, R)
    assert abs(e[0] - 1e-3) < 1e-15 and abs(e[1] - 0.1) < 1e-12
    assert oracle.rel_fro(C, R) < 1.1e-3
    # a zero row of R: the absolute error of that row
    assert oracle.row_rel_err(np.array([[0.0, 2.0]]), np.zeros((1, 2)))[0] == 2.0


# ----------------------------------------------------------------- O-7 split


def test_bf16_rne_against_torch_and_ties():
    torch = pytest.importorskip("torch")
    x = np.concatenate([si.normal_f32(3, 5000), si.row_scaled_normal_f32(4, (50, 100)).ravel(),
                        np.array([0.0, -0.0, 1.0, np.inf, -np.inf, 3.4e38, 1e-40], np.float32)])
    hi, _ = oracle.split_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(hi, ref)
    # exact ties: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7; the even
    # neighbour (1.0) wins; 1 + 3*2^-8 rounds up to the even 1 + 2^-6.
    ties = np.array([0x3F808000, 0x3F818000], dtype=np.uint32).view(np.float32)
    h, _ = oracle.split_bf16(ties)
    assert list(h) == [0x3F80, 0x3F82]


def test_bf16_split_reconstruction():
    x = si.normal_f32(9, 20000)
    hi, lo = oracle.split_bf16(x)
    rec = oracle.bf16_bits_to_f64(hi) + oracle.bf16_bits_to_f64(lo)
    # hi carries 8 significant bits, lo the next 8 (plus sign): |x - rec| <= 2^-17 |x|
    err = np.abs(rec - x.astype(np.float64))
    assert (err <= np.abs(x) * 2.0 ** -16).all()
    assert np.median(err / np.maximum(np.abs(x), 1e-30)) < 2.0 ** -17


# ---- FP16 split (O-7, fp16 form) ----------------------------------------

def test_fp16_rne_matches_library_rounding():
    # The bit-level binary16 rounding against numpy's float32 -> float16
    # conversion (round to nearest, ties to even): random values over the
    # whole fp16 range and beyond (subnormals, overflow), and exact ties.
    g = np.random.default_rng(16)
    x = (g.standard_normal(20000) * np.exp2(g.integers(-30, 20, 20000))).astype(np.float32)
    ties = [1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 2.0 ** -24 * 1.5, 2.0 ** -24 * 2.5, 65504 + 16, 2.0 ** -25]
    x = np.concatenate([x, np.array(ties, np.float32), -np.array(ties, np.float32),
                        np.array([0.0, np.inf, -np.inf, 65504, 2.0 ** -14], np.float32)])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(oracle.f32_to_fp16_bits(x), ref)
    # hand-checked ties: 1 + 2^-11 -> 1 (even), 1 + 3 * 2^-11 -> 1 + 2^-9
    assert oracle.fp16_bits_to_f64(oracle.f32_to_fp16_bits(np.array([1 + 2.0 ** -11], np.float32)))[0] == 1.0
    assert oracle.fp16_bits_to_f64(oracle.f32_to_fp16_bits(np.array([1 + 3 * 2.0 ** -11], np.float32)))[0] == \
        1 + 2.0 ** -9


def test_fp16_split_reconstructs_to_22_bits():
    # hi + lo carries 22 significant bits: |x - (hi + lo)| <= 2^-22 |x| in
    # the range the scaled operands live in.
    g = np.random.default_rng(17)
    x = (g.uniform(1, 2, 5000) * np.exp2(g.integers(-3, 14, 5000)) * g.choice([-1, 1], 5000)).astype(np.float32)
    hi, lo = oracle.split_fp16(x)
    rec = oracle.fp16_bits_to_f64(hi) + oracle.fp16_bits_to_f64(lo)
    assert np.all(np.abs(x.astype(np.float64) - rec) <= 2.0 ** -22 * np.abs(x.astype(np.float64)))
    # and hi alone is the fp16 rounding of x
    assert np.array_equal(hi, oracle.f32_to_fp16_bits(x))


def test_pow2_scales_closed_form():
    # scale = 2^(13 - floor(log2(growth * absmax))): a power of two with
    # growth * absmax * scale in [2^13, 2^14); rows of zeros keep scale 1.
    g = np.random.default_rng(18)
    amax = np.exp2(g.uniform(-40, 40, 1000))
    for growth in (1.0, 2.0, 16.0, 64.0):
        s = oracle.pow2_scales(amax, growth)
        assert np.all(np.log2(s) == np.round(np.log2(s)))
        v = growth * amax * s
        assert np.all((v >= 2.0 ** 13) & (v < 2.0 ** 14))
    assert oracle.pow2_scales(np.zeros(3), 4.0).tolist() == [1.0, 1.0, 1.0]


# ---- the split-precision product helpers (O-7) ---------------------------
#
# split3_product_f64 / split3_fp16_product_f64 are the values the GPU's
# BF16x3 / FP16x3 products are compared with.  Pinned by exact rational
# arithmetic on operands built so that the hi/lo split is known in advance:
# x = h + l with h representable in the half format and l a half-format
# value far enough below h that rounding x to the half format gives h back
# and x - h = l.  Then the helper must return exactly
# (Ah + Al)(Bh + Bl) - Al Bl = Ah Bh + Ah Bl + Al Bh, which a dropped cross
# term, an included lo*lo term or a transposed operand would all change.

from fractions import Fraction


def _bf16_pair(g, shape, e_lo=-2, e_hi=2):
    """x = h + l, h bf16 (8 significant bits) with exponent e in [e_lo, e_hi],
    l bf16 with exponent in [e - 16, e - 10]: |l| < ulp(h) / 4 and h + l
    exact in float32 (at most 24 bits from h's leading bit to l's last)."""
    e = g.integers(e_lo, e_hi + 1, shape)
    h = (128 + g.integers(0, 128, shape)) * np.exp2(e - 7.0) * g.choice([-1.0, 1.0], shape)
    f = e - g.integers(10, 17, shape)
    l = (128 + g.integers(0, 128, shape)) * np.exp2(f - 7.0) * g.choice([-1.0, 1.0], shape)
    x = (h + l).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), h + l)
    return x, h, l


def _exact_split3(Ah, Al, Bh, Bl):
    m, k = Ah.shape
    n = Bh.shape[1]
    F = np.vectorize(Fraction, otypes=[object])
    ah, al, bh, bl = F(Ah), F(Al), F(Bh), F(Bl)
    R = np.empty((m, n), dtype=object)
    for i in range(m):
        for j in range(n):
            s = Fraction(0)
            for t in range(k):
                s += (ah[i, t] + al[i, t]) * (bh[t, j] + bl[t, j]) - al[i, t] * bl[t, j]
            R[i, j] = s
    return R


def test_split3_bf16_exact_on_bf16_inputs():
    g = np.random.default_rng(31)
    A = (g.integers(-255, 256, (9, 13)) * np.exp2(g.integers(-8, 4, (9, 13)))).astype(np.float32)
    B = (g.integers(-255, 256, (13, 7)) * np.exp2(g.integers(-8, 4, (13, 7)))).astype(np.float32)
    # every entry has at most 8 significant bits: lo = 0, the helper is the product
    assert np.array_equal(oracle.split3_product_f64(A, B), A.astype(np.float64) @ B.astype(np.float64))


def test_split3_bf16_drops_exactly_the_lo_lo_term():
    g = np.random.default_rng(32)
    A, Ah, Al = _bf16_pair(g, (6, 11))
    B, Bh, Bl = _bf16_pair(g, (11, 5))
    ah, al = oracle.split_bf16(A)
    assert np.array_equal(oracle.bf16_bits_to_f64(ah), Ah) and np.array_equal(oracle.bf16_bits_to_f64(al), Al)
    got = oracle.split3_product_f64(A, B)
    want = _exact_split3(Ah, Al, Bh, Bl)
    for i in range(6):
        for j in range(5):
            assert Fraction(got[i, j]) == want[i, j], (i, j)
    # the dropped term is not negligible here: adding it changes the value
    full = (Ah + Al) @ (Bh + Bl)
    assert not np.array_equal(full, got)


def _fp16_pair_rows(g, shape, row_shift):
    """Operand whose row i, multiplied by 2^row_shift[i], is h + l with h
    fp16 (11 significant bits) and the row maximum in [2^13, 2^14) (so the
    helper's power-of-two scale for the row is exactly 2^row_shift[i]), l
    fp16 normal with exponent e - 12 or e - 13 (|l| < ulp(h) / 2, h + l exact
    in float32)."""
    r, c = shape
    e = g.integers(8, 14, shape)
    e[:, 0] = 13  # the row maximum's binade
    h = (1024 + g.integers(0, 1024, shape)) * np.exp2(e - 10.0) * g.choice([-1.0, 1.0], shape)
    f = e - g.integers(12, 14, shape)
    l = (1024 + g.integers(0, 1024, shape)) * np.exp2(f - 10.0) * g.choice([-1.0, 1.0], shape)
    s = np.exp2(-np.asarray(row_shift, dtype=np.float64))[:, None]
    x = ((h + l) * s).astype(np.float32)
    assert np.array_equal(x.astype(np.float64), (h + l) * s)
    return x, h, l


def test_split3_fp16_drops_exactly_the_lo_lo_term():
    g = np.random.default_rng(33)
    ra = g.integers(-20, 20, 5)
    cb = g.integers(-20, 20, 4)
    A, Ah, Al = _fp16_pair_rows(g, (5, 9), ra)
    Bt, Bh_t, Bl_t = _fp16_pair_rows(g, (4, 9), cb)  # B^T: its rows are B's columns
    B, Bh, Bl = Bt.T.copy(), Bh_t.T, Bl_t.T
    got = oracle.split3_fp16_product_f64(A, B)
    want = _exact_split3(Ah, Al, Bh, Bl)
    for i in range(5):
        for j in range(4):
            # A's row i is (h + l) 2^-ra[i], B's column j is (h + l) 2^-cb[j]
            w = want[i, j] * Fraction(2) ** int(-ra[i]) * Fraction(2) ** int(-cb[j])
            assert Fraction(got[i, j]) == w, (i, j)
    # lo*lo is not negligible at this size: adding it changes the value
    lolo = (Al @ Bl) * np.exp2(-ra.astype(np.float64))[:, None] * np.exp2(-cb.astype(np.float64))[None, :]
    assert np.all(lolo != 0) and not np.array_equal(got + lolo, got)


def test_split3_fp16_exact_on_fp16_inputs_and_scale_invariant():
    g = np.random.default_rng(34)
    A = g.integers(-2047, 2048, (8, 12)).astype(np.float32)
    B = g.integers(-2047, 2048, (12, 6)).astype(np.float32)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.array_equal(oracle.split3_fp16_product_f64(A, B), ref)
    # scaling row i of A by 2^e (or column j of B) scales output row i
    # (column j) by exactly 2^e, since the helper's own scale absorbs it
    A2 = A.copy()
    A2[3] *= np.float32(2.0 ** -30)
    B2 = B.copy()
    B2[:, 2] *= np.float32(2.0 ** 25)
    R = oracle.split3_fp16_product_f64(A2, B2)
    want = ref.copy()
    want[3] *= 2.0 ** -30
    want[:, 2] *= 2.0 ** 25
    assert np.array_equal(R, want)
    # and the same with lo parts present (random fp32 data)
    X = si.normal_f32(35, 8 * 12).reshape(8, 12)
    Y = si.normal_f32(36, 12 * 6).reshape(12, 6)
    P = oracle.split3_fp16_product_f64(X, Y)
    X2 = X.copy()
    X2[5] *= np.float32(2.0 ** 17)
    P2 = oracle.split3_fp16_product_f64(X2, Y)
    assert np.array_equal(P2[5], P[5] * 2.0 ** 17)
    assert np.array_equal(np.delete(P2, 5, axis=0), np.delete(P, 5, axis=0))


# ---- Strassen layouts: SAR-Strassen, STAR-Strassen-2 (space) ----------------


@pytest.mark.parametrize("variant", [oracle.STRASSEN_CLASSIC, oracle.STRASSEN_WINOGRAD])
def test_strassen_layout_exact_over_z_every_layout(variant):
    g = np.random.default_rng(41 + variant)
    for depth in range(4):
        for layout in range(1 << depth):
            for (m, k, n) in [(37, 29, 41), (16, 16, 16), (9, 1, 5), (64, 33, 2)]:
                A = g.integers(-300, 300, (m, k))
                B = g.integers(-300, 300, (k, n))
                C0 = g.integers(-300, 300, (m, n))
                C, _ = oracle.strassen_layout(A, B, depth, variant, layout, C0)
                assert np.array_equal(C, C0 + A @ B), (depth, layout, m, k, n)


def test_strassen_layout_float_close_and_order_independent():
    # float64: every layout evaluates the same products and sums; error
    # against the float64 product stays at Strassen's level
    A = si.normal_f32(43, (96, 80)).astype(np.float64)
    B = si.normal_f32(44, (80, 72)).astype(np.float64)
    ref = A @ B
    for layout in range(8):
        C, _ = oracle.strassen_layout(A, B, 3, oracle.STRASSEN_WINOGRAD, layout)
        assert oracle.rel_fro(C, ref) < 1e-13


def _closed_form_peak(n, depth, k_bf, per_level):
    """k_bf breadth-first levels on top (per_level temporaries each), the
    rest depth-first (3 each), every breadth-first sub-product concurrent."""
    s = sum(7 ** j * per_level * (n >> (j + 1)) ** 2 for j in range(k_bf))
    s += 7 ** k_bf * 3 * sum((n >> j) ** 2 for j in range(k_bf + 1, depth + 1))
    return s


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_layout_space_closed_forms(depth):
    n = 64
    A = np.ones((n, n), np.int64)
    per = GOLD["strassen_straightforward_temps_per_level"]["value"]
    sar = GOLD["sar_strassen_temps_per_depth"]["value"]
    assert (per, sar) == (17, 3)
    # _closed_form_peak is the printed STAR-Strassen-2 space formula
    assert GOLD["star_strassen_2_space"]["formula"].startswith("sum_{j<k} 7^j 17 (n/2^(j+1))^2 + 7^k * 3")
    for k_bf in range(depth + 1):
        # bits of the depth-first levels: k_bf .. depth - 1
        layout = ((1 << depth) - 1) & ~((1 << k_bf) - 1)
        _, peak = oracle.strassen_layout(A, A, depth, oracle.STRASSEN_CLASSIC, layout)
        assert peak == _closed_form_peak(n, depth, k_bf, per), (depth, k_bf)
    # SAR-Strassen at every depth: 3 (n/2)^2 + 3 (n/4)^2 + ... < n^2, the
    # limit the paper solves the recurrence to
    _, peak = oracle.strassen_layout(A, A, depth, oracle.STRASSEN_CLASSIC, (1 << depth) - 1)
    assert peak == 3 * sum((n >> j) ** 2 for j in range(1, depth + 1))
    assert peak < GOLD["sar_strassen_temps_per_depth"]["limit_in_n2"] * n * n
    # Strassen-Winograd's level holds 4 + 4 operand sums and 7 products
    _, peak = oracle.strassen_layout(A, A, 1, oracle.STRASSEN_WINOGRAD, 0)
    assert peak == 15 * (n // 2) ** 2
