"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host planner (no HIP call) validates arguments and sizes the workspace as
the paper's space recurrences say.  No compute call is made here."""
import ctypes
import json
import os
import re

import pytest

import paper_1911_05328_amd as sm
from paper_1911_05328_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "closed_forms.json")))
MiB = 1 << 20


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(mm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert {"mm_semiring", "mm_strassen", "mm_plan", "mm_status_string"} <= set(names)
    for nm in names:
        assert hasattr(L, nm), nm


def test_status_strings():
    for st in (0, -1, -2, -3, -4):
        assert _lib.status_string(st)
    assert _lib.lib().mm_version() >= 100


def test_plan_default_min_plus_4096():
    st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, 4096, 4096, 4096, 0)
    assert st == sm.MM_OK
    assert p["sched"]["split_k"] == 1 and p["ws_bytes"] == 0
    assert p["tiles_m"] * p["tiles_n"] * p["sched"]["split_k"] == p["workgroups"]


@pytest.mark.parametrize("budget,expect_s", [(64 * MiB, 2), (128 * MiB, 2), (256 * MiB, 4)])
def test_split_at_budget_whole_c(budget, expect_s):
    # One band of all rows: (s - 1) n^2 int32 temporaries must fit the budget.
    n = 4096
    best = None
    for s in (1, 2, 4, 8):
        st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, budget,
                        sm.make_schedule(tile=128, split_k=s, band_rows=n))
        if st == sm.MM_OK:
            assert p["ws_bytes"] == (s - 1) * n * n * 4 <= budget
            best = s
    assert best == expect_s


@pytest.mark.parametrize("j", [1, 2, 3])
def test_temp_count_matches_top_level_split_closed_form(j):
    # Temporaries at the top j recursion levels: (2^j - 1) n^2 elements.
    n = 1024
    st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 1 << 40,
                    sm.make_schedule(tile=64, split_k=2 ** j, band_rows=n))
    assert st == sm.MM_OK
    assert p["temp_elems"] == (2 ** j - 1) * n * n
    assert p["sar_levels"] == j and p["tar_levels"] == 0


def test_tar_levels_need_no_temporaries():
    n = 2048
    st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 0, sm.make_schedule(tile=128, split_k=8, star_depth=3))
    assert st == sm.MM_OK and p["ws_bytes"] == 0 and p["tar_levels"] == 3
    # STAR: one TAR level above two SAR levels: 2 groups x 3 temporaries.
    st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 1 << 40,
                    sm.make_schedule(tile=128, split_k=8, star_depth=1, band_rows=n))
    assert st == sm.MM_OK and p["temp_elems"] == 2 * 3 * n * n


def test_banding_bounds_space_by_band():
    # s = 4 under a 1x n^2 budget: the planner chooses bands whose three
    # temporaries fit, instead of refusing.
    n = 4096
    st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 64 * MiB, sm.make_schedule(tile=128, split_k=4))
    assert st == sm.MM_OK
    assert p["ws_bytes"] <= 64 * MiB
    band = p["sched"]["band_rows"]
    assert band % 128 == 0 and band * 3 * n * 4 <= 64 * MiB
    assert p["bands"] == -(-n // band)


def test_explicit_schedule_that_does_not_fit_is_rejected():
    n = 4096
    st, _ = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 64 * MiB,
                    sm.make_schedule(tile=128, split_k=4, band_rows=n))
    assert st == sm.MM_ERR_WORKSPACE
    # not even one band row of temporaries fits
    st, _ = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 1024, sm.make_schedule(tile=128, split_k=2))
    assert st == sm.MM_ERR_WORKSPACE


def test_planner_split_counts_rounds_of_wide_tiles():
    # One 256 tile per CU: the planner's split takes the fewest whole rounds
    # of 256 workgroups per unit of k.  195 tiles fill one round unsplit;
    # splitting would add rounds as fast as it shortens them.
    GiB = 1 << 30
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_BF16, 3247, 3735, 2342, GiB, sm.make_schedule(tile=256))
    assert st == sm.MM_OK and p["sched"]["split_k"] == 1
    # 100 tiles: two slices each still fit one round
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_BF16, 2560, 2560, 4096, GiB, sm.make_schedule(tile=256))
    assert st == sm.MM_OK and p["sched"]["split_k"] == 2 and p["workgroups"] <= 256
    # 4 tiles and a deep k: split until the slices fill a round or reach 16 k-blocks each
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_BF16, 512, 512, 65536, GiB, sm.make_schedule(tile=256))
    assert st == sm.MM_OK and p["sched"]["split_k"] == 64 and p["workgroups"] == 256
    # smaller tiles keep the fill rule (split while under two workgroups per CU)
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_BF16, 2560, 2560, 4096, GiB, sm.make_schedule(tile=128))
    assert st == sm.MM_OK and p["sched"]["split_k"] == 2


EMPTY_SHAPES = [(0, 64, 64), (64, 0, 64), (64, 64, 0), (0, 0, 0)]


@pytest.mark.parametrize("shape", EMPTY_SHAPES)
def test_empty_products_need_no_workspace(shape):
    # An empty product launches nothing: every valid schedule plans with no
    # workspace, k-splits, Strassen levels, FP16x3 and the slot ring included.
    cases = [(sm.PLUS_TIMES, sm.DT_F32, s) for s in (
        None, sm.make_schedule(tile=128, split_k=4), sm.make_schedule(strassen_depth=2, precision=sm.PREC_BF16X3),
        sm.make_schedule(precision=sm.PREC_FP16X3), sm.make_schedule(tile=64, split_k=4, star_depth=1,
                                                                      flags=sm.FLAG_NONDETERMINISTIC))]
    cases += [(sm.PLUS_TIMES, dt, s) for dt in (sm.DT_BF16, sm.DT_F16)
              for s in (None, sm.make_schedule(tile=256, split_k=2), sm.make_schedule(tile=128))]
    cases += [(sm.MIN_PLUS, sm.DT_I32, s) for s in (
        None, sm.make_schedule(tile=128, split_k=8), sm.make_schedule(tile=128, split_k=8, star_depth=2),
        sm.make_schedule(tile=128, split_k=8, flags=sm.FLAG_PERSISTENT))]
    for sr, dt, s in cases:
        st, p = sm.plan(sr, dt, *shape, 0, s)
        assert st == sm.MM_OK and p["ws_bytes"] == 0, (sr, dt, shape, st)
    m, n, k = shape
    for depth in (0, 1, 2):
        for prec in (sm.PREC_BF16X3, sm.PREC_FP16X3):
            assert sm.strassen_workspace_bytes(m, n, k, depth, sm.CLASSIC, prec) == 0
    # the calls themselves return before touching the device (dummy pointers
    # stand for the operands of the non-empty sides)
    L = _lib.lib()
    P = ctypes.c_void_p(4096)
    for depth in (0, 1, 2):
        assert L.mm_strassen(m, n, k, P, max(k, 1), P, max(n, 1), P, max(n, 1), depth, 0, sm.PREC_BF16X3, None, 0,
                             None) == sm.MM_OK
    assert L.mm_semiring(sm.MIN_PLUS, sm.DT_I32, m, n, k, P, max(k, 1), P, max(n, 1), P, max(n, 1), None, 0,
                         ctypes.byref(sm.make_schedule(tile=128, split_k=8)), None) == sm.MM_OK


def test_misaligned_workspace_is_refused_before_any_launch():
    # every entry point that takes a caller workspace refuses one that does
    # not start on a 256-byte boundary (its sub-buffers sit at 256-byte
    # offsets and are read with 16-byte and direct-to-LDS loads)
    L = _lib.lib()
    P = ctypes.c_void_p(1 << 20)
    bad = ctypes.c_void_p((1 << 20) + 16)
    big = 1 << 30
    s = sm.make_schedule(tile=128, split_k=4)
    assert L.mm_semiring(sm.MIN_PLUS, sm.DT_I32, 256, 256, 256, P, 256, P, 256, P, 256, bad, big,
                         ctypes.byref(s), None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_strassen(256, 256, 256, P, 256, P, 256, P, 256, 1, 0, sm.PREC_BF16X3, bad, big,
                         None) == sm.MM_ERR_INVALID_ARG
    sc = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
    assert L.mm_bilinear(256, 256, 256, P, 256, P, 256, P, 256, ctypes.byref(sc), sm.PREC_BF16X3, bad, big,
                         None) == sm.MM_ERR_INVALID_ARG
    prob = (_lib.Problem * 1)()
    prob[0] = _lib.Problem(64, 64, 64, 1 << 20, 64, 1 << 20, 64, 1 << 20, 64)
    assert L.mm_batched(1, prob, sm.DT_BF16, None, bad, big, None) == sm.MM_ERR_INVALID_ARG
    g = ctypes.c_void_p()
    assert L.mm_batched_graph_create(1, prob, sm.DT_BF16, None, bad, big, None, ctypes.byref(g)) == \
        sm.MM_ERR_INVALID_ARG


def test_planner_falls_back_without_budget():
    # Skinny product that wants a k-split: with no workspace the exact
    # semiring uses TAR merging, the float path drops the split.
    st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, 256, 256, 65536, 0)
    assert st == sm.MM_OK and p["sched"]["split_k"] > 1 and p["ws_bytes"] == 0
    assert p["tar_levels"] == p["tar_levels"] + p["sar_levels"]
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, 256, 256, 65536, 0)
    assert st == sm.MM_OK and p["sched"]["split_k"] == 1
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, 256, 256, 65536, 1 << 30)
    assert st == sm.MM_OK and p["sched"]["split_k"] > 1 and 0 < p["ws_bytes"] <= 1 << 30


@pytest.mark.parametrize("args,expect", [
    ((sm.MIN_PLUS, sm.DT_F32), sm.MM_ERR_UNSUPPORTED),
    ((sm.MAX_MIN, sm.DT_F32), sm.MM_ERR_UNSUPPORTED),
    ((sm.OR_AND, sm.DT_BF16), sm.MM_ERR_UNSUPPORTED),
    ((sm.PLUS_TIMES, sm.DT_I32), sm.MM_ERR_UNSUPPORTED),
    ((5, sm.DT_I32), sm.MM_ERR_INVALID_ARG),
    ((7, sm.DT_I32), sm.MM_ERR_INVALID_ARG),
    ((sm.MIN_PLUS, 9), sm.MM_ERR_INVALID_ARG),
])
def test_bad_combinations(args, expect):
    st, _ = sm.plan(args[0], args[1], 64, 64, 64, 0)
    assert st == expect


def test_strassen_on_non_ring_is_unsupported():
    # Strassen needs the additive inverse: (min,+), (max,+), (max, min) and
    # Boolean (or, and) have none.
    for sr in (sm.MIN_PLUS, sm.MAX_PLUS, sm.MAX_MIN, sm.OR_AND):
        st, _ = sm.plan(sr, sm.DT_I32, 64, 64, 64, 0, sm.make_schedule(strassen_depth=1))
        assert st == sm.MM_ERR_UNSUPPORTED


@pytest.mark.parametrize("sched", [
    dict(split_k=3), dict(split_k=128), dict(tile=48), dict(split_k=4, star_depth=3),
    dict(band_rows=100, tile=64), dict(flags=16), dict(split_k=-1),
])
def test_bad_schedules(sched):
    st, _ = sm.plan(sm.MIN_PLUS, sm.DT_I32, 512, 512, 512, 1 << 30, sm.make_schedule(**sched))
    assert st == sm.MM_ERR_INVALID_ARG


def test_float_atomic_merge_needs_flag():
    s = sm.make_schedule(split_k=4, star_depth=2)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, 512, 512, 4096, 0, s)[0] == sm.MM_ERR_INVALID_ARG
    s = sm.make_schedule(split_k=4, star_depth=2, flags=sm.FLAG_NONDETERMINISTIC)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, 512, 512, 4096, 0, s)[0] == sm.MM_OK


def test_negative_and_empty_sizes():
    assert sm.plan(sm.MIN_PLUS, sm.DT_I32, -1, 4, 4, 0)[0] == sm.MM_ERR_INVALID_ARG
    for dims in ((0, 5, 5), (5, 0, 5), (5, 5, 0)):
        assert sm.plan(sm.MIN_PLUS, sm.DT_I32, *dims, 0)[0] == sm.MM_OK


def test_mm_semiring_validates_before_launch():
    # Invalid leading dimensions and null pointers are refused on the host,
    # so these calls never reach the GPU (there is none here).
    L = _lib.lib()
    p = ctypes.c_void_p(16)
    assert L.mm_semiring(1, 0, 4, 4, 4, p, 3, p, 4, p, 4, None, 0, None, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_semiring(1, 0, 4, 4, 4, None, 4, p, 4, p, 4, None, 0, None, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_semiring(1, 0, 4, 4, 4, p, 4, p, 4, p, 4, None, 64, None, None) == sm.MM_ERR_INVALID_ARG
    # empty problems succeed without touching memory
    assert L.mm_semiring(1, 0, 0, 4, 4, None, 4, p, 4, None, 4, None, 0, None, None) == sm.MM_OK


# ------------------------------------------------------------ Strassen (host)

def strassen_tables(variant):
    import numpy as np
    a = (ctypes.c_int8 * 28)()
    b = (ctypes.c_int8 * 28)()
    g = (ctypes.c_int8 * 28)()
    assert _lib.lib().mm_strassen_coefficients(variant, a, b, g) == sm.MM_OK
    return (np.array(a, dtype=np.int64).reshape(7, 2, 2), np.array(b, dtype=np.int64).reshape(7, 2, 2),
            np.array(g, dtype=np.int64).reshape(7, 2, 2))


@pytest.mark.parametrize("variant", [sm.CLASSIC, sm.WINOGRAD])
def test_device_strassen_tables_are_the_2x2x2_product(variant):
    # The library's coefficient tables must reproduce the 2x2x2 matrix
    # multiplication tensor: sum_r alpha_r[a,b] beta_r[c,d] gamma_r[e,f]
    # = [b == c][a == e][d == f] for all 64 index combinations.
    import itertools
    al, be, ga = strassen_tables(variant)
    for a, b, c, d, e, f in itertools.product(range(2), repeat=6):
        t = sum(al[r, a, b] * be[r, c, d] * ga[r, e, f] for r in range(7))
        assert t == int(b == c and a == e and d == f), (a, b, c, d, e, f)


def test_classic_table_is_the_printed_one_and_temp_count():
    # Classic: the products exactly as printed (P1 = (A00+A11)(B00+B11), ...).
    # Operands that are a bare quadrant (S3 = A00, S4 = A11, T2 = B00,
    # T5 = B11) need no temporary in the straightforward parallel Strassen, so
    # it holds 17 = 7 products + 10 formed operands per level (Lemma
    # par-strassen).  This library's breadth-first layout copies those four
    # as well: 21 leaf-sized buffers at depth 1.
    import numpy as np
    al, be, ga = strassen_tables(sm.CLASSIC)
    assert al[0].tolist() == [[1, 0], [0, 1]] and be[0].tolist() == [[1, 0], [0, 1]]
    assert ga[:, 0, 0].tolist() == [1, 0, 0, 1, -1, 0, 1]   # C00 = P1 + P4 - P5 + P7
    bare = sum(int(np.count_nonzero(x[r]) == 1) for x in (al, be) for r in range(7))
    assert bare == 4
    assert 7 + (14 - bare) == GOLD["strassen_straightforward_temps_per_level"]["value"]
    n = 1024
    ws = sm.strassen_workspace_bytes(n, n, n, 1, sm.CLASSIC, sm.PREC_F32)
    assert ws == 21 * (n // 2) ** 2 * 4
    # BF16x3: the leaf operands as bf16 hi/lo planes (same bytes as fp32;
    # B is read in place for the B^T leaves): 7 + 7 + 7 products
    ws = sm.strassen_workspace_bytes(n, n, n, 1, sm.CLASSIC, sm.PREC_BF16X3)
    assert ws == 21 * (n // 2) ** 2 * 4


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_workspace_and_plan(depth):
    m, n, k = 1000, 777, 1500
    s = sm.make_schedule(strassen_depth=depth, precision=sm.PREC_BF16X3, tile=64, split_k=2)
    need = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, need, s)
    assert st == sm.MM_OK and p["leaves"] == 7 ** depth
    hm, hn, hk = m, n, k
    for _ in range(depth):
        hm, hn, hk = -(-hm // 2), -(-hn // 2), -(-hk // 2)
    assert (p["leaf_m"], p["leaf_n"], p["leaf_k"]) == (hm, hn, hk)
    assert p["sched"]["strassen_layout"] == sm.strassen_layout(0)  # every level breadth-first
    # the same levels explicitly breadth-first do not fit one byte less ...
    bf = sm.make_schedule(strassen_depth=depth, precision=sm.PREC_BF16X3, tile=64, split_k=2,
                          strassen_layout=sm.strassen_layout(0))
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, need - 1, bf)[0] == sm.MM_ERR_WORKSPACE
    # ... while the planner then makes the top level depth-first
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, need - 1, s)
    assert st == sm.MM_OK and p["sched"]["strassen_layout"] == sm.strassen_layout(1)
    # every level depth-first is the least workspace; below it nothing fits
    sar = sm.make_schedule(strassen_depth=depth, precision=sm.PREC_BF16X3, tile=64, split_k=2,
                           strassen_layout=sm.strassen_layout((1 << depth) - 1))
    least = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, sar)
    assert 0 < least < need
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, least - 1, s)[0] == sm.MM_ERR_WORKSPACE
    # the public mm_strassen refuses a workspace below that before touching the GPU
    L = _lib.lib()
    p16 = ctypes.c_void_p(256)
    short = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, sm.make_schedule(
        strassen_depth=depth, precision=sm.PREC_BF16X3, variant=sm.WINOGRAD, tile=0, split_k=1,
        strassen_layout=sm.strassen_layout((1 << depth) - 1))) - 1
    assert L.mm_strassen(m, n, k, p16, k, p16, n, p16, n, depth, sm.WINOGRAD, sm.PREC_BF16X3,
                         p16, short, None) == sm.MM_ERR_WORKSPACE


@pytest.mark.parametrize("prec", [sm.PREC_F32, sm.PREC_BF16X3])
@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_depth_first_levels_workspace_closed_forms(prec, depth):
    # n = 1024 square, leaves h = n / 2^depth (whole 32-row plane units, no
    # padding), one k-slice: a round with t depth-first levels on top holds
    # the 7^(depth - t) leaves of the breadth-first levels below, each as an
    # A operand, a B operand and a product (4 bytes per element, hi + lo
    # planes included).  All levels breadth-first: 3 * 7^depth leaf-size
    # buffers (21 at depth 1: the printed variant's 17 temporaries of Lemma
    # par-strassen plus the 4 bare-quadrant operands copied for uniform leaf
    # products); all depth-first: 3 leaf-size buffers whatever the depth,
    # at most the 3 per depth of Lemma sar-strassen, since S_r, T_r are
    # formed straight from A and B and P_r is added into C at once.
    n = 1024
    h = n >> depth
    for t in range(depth + 1):
        s = sm.make_schedule(strassen_depth=depth, precision=prec, variant=sm.CLASSIC, tile=128, split_k=1,
                             strassen_layout=sm.strassen_layout((1 << t) - 1))
        ws = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, n, n, n, s)
        assert ws == 3 * 7 ** (depth - t) * h * h * 4, (t, ws)
        st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, n, n, n, ws, s)
        assert st == sm.MM_OK and p["leaves"] == 7 ** depth
        assert p["workgroups"] == (h // 128) ** 2 * 7 ** (depth - t)  # one round's leaf launch
    assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, n, n, n, sm.make_schedule(
        strassen_depth=depth, precision=prec, tile=128, split_k=1,
        strassen_layout=sm.strassen_layout((1 << depth) - 1))) <= 3 * sum((n >> l) ** 2 for l in range(1, depth + 1)) * 4


def test_strassen_layout_rules():
    m = n = k = 512
    base = dict(strassen_depth=2, precision=sm.PREC_BF16X3)
    # bits beyond the depth, or without the "given" bit: invalid
    for bad in (sm.strassen_layout(4), 1, 3):
        st, _ = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, 1 << 30, sm.make_schedule(strassen_layout=bad, **base))
        assert st == sm.MM_ERR_INVALID_ARG, bad
    # depth-first levels below a breadth-first one are not built
    st, _ = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, 1 << 30,
                    sm.make_schedule(strassen_layout=sm.strassen_layout(2), **base))
    assert st == sm.MM_ERR_UNSUPPORTED
    # a layout on a schedule without Strassen levels
    st, _ = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, 1 << 30,
                    sm.make_schedule(precision=sm.PREC_BF16X3, strassen_layout=sm.strassen_layout(1)))
    assert st == sm.MM_ERR_INVALID_ARG
    for ok_layout in (0, sm.strassen_layout(0), sm.strassen_layout(1), sm.strassen_layout(3)):
        st, _ = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, 1 << 30, sm.make_schedule(strassen_layout=ok_layout, **base))
        assert st == sm.MM_OK, ok_layout


def test_bf16x3_planes_need_workspace_and_flag_disables_them():
    m, n, k = 1000, 900, 777
    s = sm.make_schedule(tile=128, split_k=1, precision=sm.PREC_BF16X3)
    ldp = -(-k // 32) * 32  # plane rows: whole 32-deep k-tiles, zero-padded
    rows = -(-m // 32) * 32 + -(-n // 32) * 32  # whole 32-row units per plane
    planes = -(-(rows * ldp * 4) // 256) * 256
    assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s) == planes
    st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, planes - 1, s)
    assert st == sm.MM_OK and p["ws_bytes"] == 0  # falls back to the in-kernel split
    s2 = sm.make_schedule(tile=128, split_k=1, precision=sm.PREC_BF16X3, flags=sm.FLAG_SPLIT_IN_KERNEL)
    assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s2) == 0


def test_fp16x3_workspace_closed_form_and_schedule_rules():
    # FP16x3 holds the same planes as BF16x3 (fp16 hi/lo instead of bf16)
    # plus the scale region: |A| row maxima, |B| column maxima (each padded
    # to 64 floats) and a scale and its inverse per leaf row / column
    # (whole 32-row units), 256-byte aligned.
    r32 = lambda x: -(-x // 32) * 32  # noqa: E731
    r64 = lambda x: -(-x // 64) * 64  # noqa: E731
    r256 = lambda x: -(-x // 256) * 256  # noqa: E731
    m, n, k = 1000, 900, 777
    for depth in (0, 1, 2):
        hm, hn = m, n
        for _ in range(depth):
            hm, hn = -(-hm // 2), -(-hn // 2)
        scales = r256(4 * (r64(m) + r64(n) + 2 * r32(hm) + 2 * r32(hn)))
        for variant in (sm.CLASSIC, sm.WINOGRAD):
            b = sm.strassen_workspace_bytes(m, n, k, depth, variant, sm.PREC_BF16X3)
            f = sm.strassen_workspace_bytes(m, n, k, depth, variant, sm.PREC_FP16X3)
            assert f == r256(b) + scales, (depth, variant)
            assert sm.strassen_workspace_bytes(m, n, k, depth, variant, sm.PREC_FP16X3_HIACC) == f
    # through mm_semiring at depth 0: the same orchestration, planes always
    s = sm.make_schedule(tile=128, split_k=1, precision=sm.PREC_FP16X3)
    need = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
    assert need == sm.strassen_workspace_bytes(m, n, k, 0, sm.WINOGRAD, sm.PREC_FP16X3)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, need - 1, s)[0] == sm.MM_ERR_WORKSPACE
    # no in-kernel split, no banding, at most 3 8-way levels above (star_depth
    # counts those here, not TAR merges), no bf16 inputs, no (min,+)
    for bad in (dict(flags=sm.FLAG_SPLIT_IN_KERNEL),
                dict(split_k=2, star_depth=4),
                dict(band_rows=128)):
        s = sm.make_schedule(tile=128, precision=sm.PREC_FP16X3, **bad)
        assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, 1 << 40, s)[0] == sm.MM_ERR_INVALID_ARG, bad
    s = sm.make_schedule(precision=sm.PREC_FP16X3)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_BF16, m, n, k, 1 << 40, s)[0] == sm.MM_ERR_INVALID_ARG
    assert sm.plan(sm.MIN_PLUS, sm.DT_I32, m, n, k, 1 << 40, s)[0] == sm.MM_ERR_INVALID_ARG
    # precisions past the last one are rejected everywhere
    s = sm.make_schedule(precision=6)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, 1 << 40, s)[0] == sm.MM_ERR_INVALID_ARG
    assert sm.strassen_workspace_bytes(m, n, k, 1, sm.WINOGRAD, 6) == 0


def test_f16_inputs_plan_rules():
    # fp16 inputs: one fp16 product (precision F32 = native), tiles up to 256,
    # k-split temporaries as for bf16 inputs; no split precision, no
    # Strassen levels, no integer semiring.
    m, n, k = 1000, 900, 777
    for tile in (32, 64, 128, 256):
        s = sm.make_schedule(tile=tile, split_k=2)
        st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F16, m, n, k, 1 << 40, s)
        assert st == sm.MM_OK and p["tile_k"] == 32
        assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F16, m, n, k, s) == \
            sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_BF16, m, n, k, s)
    # 128- and 256-wide tiles copy both operands once into one 16-bit plane
    # each (rows rounded up to 32, k to 32, B transposed) when the budget
    # holds them; narrower tiles, MM_FLAG_SPLIT_IN_KERNEL or a budget
    # without room stage straight from the operands
    ldp = -(-k // 32) * 32
    planes = -(-((-(-m // 32) * 32 + -(-n // 32) * 32) * ldp * 2) // 256) * 256
    for dt in (sm.DT_F16, sm.DT_BF16):
        for tile in (32, 64, 128, 256):
            s = sm.make_schedule(tile=tile, split_k=1)
            st, p = sm.plan(sm.PLUS_TIMES, dt, m, n, k, 1 << 40, s)
            assert st == sm.MM_OK and p["ws_bytes"] == (planes if tile >= 128 else 0), (dt, tile)
            s_ik = sm.make_schedule(tile=tile, split_k=1, flags=sm.FLAG_SPLIT_IN_KERNEL)
            assert sm.plan(sm.PLUS_TIMES, dt, m, n, k, 1 << 40, s_ik)[1]["ws_bytes"] == 0
            assert sm.plan(sm.PLUS_TIMES, dt, m, n, k, planes - 1, s)[1]["ws_bytes"] == 0
    for prec in (sm.PREC_BF16X3, sm.PREC_BF16, sm.PREC_FP16X3):
        s = sm.make_schedule(precision=prec)
        assert sm.plan(sm.PLUS_TIMES, sm.DT_F16, m, n, k, 1 << 40, s)[0] == sm.MM_ERR_INVALID_ARG, prec
    s = sm.make_schedule(strassen_depth=1)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F16, m, n, k, 1 << 40, s)[0] == sm.MM_ERR_UNSUPPORTED
    assert sm.plan(sm.MIN_PLUS, sm.DT_F16, m, n, k, 1 << 40, None)[0] == sm.MM_ERR_UNSUPPORTED
    assert sm.plan(sm.PLUS_TIMES, 4, m, n, k, 1 << 40, None)[0] == sm.MM_ERR_INVALID_ARG


@pytest.mark.parametrize("sr", [sm.MAX_MIN, sm.OR_AND])
def test_exact_semirings_plan_like_minplus(sr):
    # (max, min) and Boolean are exact like (min,+): the same tiles, split
    # temporaries and budget fallback to TAR merging (no temporaries).
    for budget in (0, 1 << 20, 1 << 30):
        a = sm.plan(sm.MIN_PLUS, sm.DT_I32, 4096, 4096, 4096, budget)
        b = sm.plan(sr, sm.DT_I32, 4096, 4096, 4096, budget)
        assert a == b
    s = sm.make_schedule(split_k=4, star_depth=2)
    assert sm.plan(sr, sm.DT_I32, 512, 512, 4096, 0, s)[0] == sm.MM_OK


@pytest.mark.parametrize("prec", [sm.PREC_F32, sm.PREC_BF16X3, sm.PREC_FP16X3])
def test_star_strassen_workspace_is_that_of_the_largest_sub_product(prec):
    # STAR-Strassen (8-way levels above the Strassen levels): the workspace
    # is one Strassen workspace of the first (largest, ceil-halved) block,
    # reused by all 8^t sub-products; no flag needed (serialised, ordered).
    m, n, k = 1000, 777, 1500
    for t in (1, 2, 3):
        for depth in (1, 2):
            s = sm.make_schedule(strassen_depth=depth, star_depth=t, variant=sm.WINOGRAD, precision=prec,
                                 tile=128, split_k=1)
            need = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s)
            hm, hn, hk = m, n, k
            for _ in range(t):
                hm, hn, hk = -(-hm // 2), -(-hn // 2), -(-hk // 2)
            s0 = sm.make_schedule(strassen_depth=depth, variant=sm.WINOGRAD, precision=prec, tile=128, split_k=1)
            assert need == sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, hm, hn, hk, s0), (t, depth)
            assert need < sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, m, n, k, s0)
            st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, need, s)
            assert st == sm.MM_OK and p["leaves"] == 8 ** t * 7 ** depth and p["tar_levels"] == t
            s_bf = sm.make_schedule(strassen_depth=depth, star_depth=t, variant=sm.WINOGRAD, precision=prec,
                                    tile=128, split_k=1, strassen_layout=sm.strassen_layout(0))
            assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, m, n, k, need - 1, s_bf)[0] == sm.MM_ERR_WORKSPACE


@pytest.mark.parametrize("prec", [sm.PREC_F32, sm.PREC_BF16X3])
def test_star_strassen_1_temporaries_within_the_papers_n2(prec):
    # Thm. star-strassen-1: besides the 3 n^2 of A, B and C (what CO2 holds,
    # and all it holds: no workspace), STAR-Strassen needs 1 n^2 of
    # temporaries.  The TAR levels on top need none (each C quadrant takes
    # its k-halves in order), and with the Strassen levels of the
    # (n / 2^t)-sized sub-products depth-first the workspace is 3 leaf-size
    # buffers reused by every sub-product: 3 (n / 2^(t + d))^2 <= n^2.  With
    # them breadth-first (the planner's choice when the workspace holds it,
    # and faster) it is 3 * 7^d leaf-size buffers, 21/16 n^2 at t = d = 1:
    # above the paper's bound, which the depth-first layout meets.
    bound = GOLD["star_strassen_1_extra_space"]["value_in_n2"]
    assert bound == 1 and GOLD["co2_io_space"]["value_in_n2"] == 3
    n = 1024
    assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, n, n, n, sm.make_schedule(tile=128, split_k=1)) == 0
    for t in (1, 2):
        for d in (1, 2):
            h = n >> (t + d)
            common = dict(strassen_depth=d, star_depth=t, precision=prec, variant=sm.CLASSIC, tile=128, split_k=1)
            df = sm.make_schedule(strassen_layout=sm.strassen_layout((1 << d) - 1), **common)
            ws = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, n, n, n, df)
            assert ws == 3 * h * h * 4 and ws <= bound * n * n * 4, (t, d, ws)
            st, p = sm.plan(sm.PLUS_TIMES, sm.DT_F32, n, n, n, ws, df)
            assert st == sm.MM_OK and p["leaves"] == 8 ** t * 7 ** d and p["tar_levels"] == t
            bf = sm.make_schedule(strassen_layout=sm.strassen_layout(0), **common)
            assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, n, n, n, bf) == 3 * 7 ** d * h * h * 4, (t, d)
    bf = sm.make_schedule(strassen_depth=1, star_depth=1, precision=prec, variant=sm.CLASSIC, tile=128, split_k=1,
                          strassen_layout=sm.strassen_layout(0))
    assert sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, n, n, n, bf) * 16 == 21 * n * n * 4


def _tile_order(tm, tn):
    import numpy as np
    ti = np.zeros(max(tm * tn, 1), dtype=np.int64)
    tj = np.zeros(max(tm * tn, 1), dtype=np.int64)
    P = ctypes.POINTER(ctypes.c_int64)
    st = _lib.lib().mm_tile_order(tm, tn, ti.ctypes.data_as(P), tj.ctypes.data_as(P))
    assert st == sm.MM_OK
    return ti[: tm * tn], tj[: tm * tn]


def test_tile_order_is_a_permutation_and_morton_on_square_grids():
    import numpy as np
    # every tile exactly once, for all small grids and some long thin ones
    shapes = [(a, b) for a in range(1, 41) for b in range(1, 41)]
    shapes += [(64, 2), (3, 100), (1000, 7), (1, 513), (257, 129)]
    for tm, tn in shapes:
        ti, tj = _tile_order(tm, tn)
        assert (ti >= 0).all() and (ti < tm).all() and (tj >= 0).all() and (tj < tn).all()
        assert len(set(zip(ti.tolist(), tj.tolist()))) == tm * tn, (tm, tn)
    # square power-of-two grids: the quadrant (Morton) order, i.e. bits of
    # t alternate between the row and the column index, row bit first
    for L in (1, 2, 3, 5):
        s = 1 << L
        ti, tj = _tile_order(s, s)
        for t in range(s * s):
            i = sum(((t >> (2 * b + 1)) & 1) << b for b in range(L))
            j = sum(((t >> (2 * b)) & 1) << b for b in range(L))
            assert (ti[t], tj[t]) == (i, j)
    # a 64 x 4 grid is halved along its rows until square: the first 16
    # tiles are the top 4 x 4 block
    ti, tj = _tile_order(64, 4)
    assert set(zip(ti[:16].tolist(), tj[:16].tolist())) == {(i, j) for i in range(4) for j in range(4)}
    ti, tj = _tile_order(4, 64)
    assert set(zip(ti[:16].tolist(), tj[:16].tolist())) == {(i, j) for i in range(4) for j in range(4)}
    assert _lib.lib().mm_tile_order(-1, 3, None, None) == sm.MM_ERR_INVALID_ARG
    assert _lib.lib().mm_tile_order(0, 5, None, None) == sm.MM_OK


def test_persistent_plan_workspace_is_independent_of_size():
    # MM_FLAG_PERSISTENT: a control block (16 bytes + 12 per slot group,
    # 256-aligned) and min(PERSIST_SLOTS / split_k, tiles) groups of split_k
    # tile-sized int32 slots -- the paper's min{p, 4^d} blocks per depth
    # (a fixed number of slots, or one per block when there are fewer
    # blocks) -- whatever k is, and independent of m, n once the tiles
    # outnumber the ring.
    assert GOLD["sar_blocks_per_depth"]["formula"] == "min(p, 4^d)"
    r256 = lambda x: -(-x // 256) * 256  # noqa: E731
    for tile in (32, 64, 128):
        for s in (1, 2, 4, 64):
            for n in (100, 4096, 65536):
                tiles = (-(-n // tile)) ** 2
                groups = min(-(-sm.PERSIST_SLOTS // s), tiles) if s > 1 else 0
                expect = r256(16 + 12 * groups) + groups * s * tile * tile * 4
                if n >= 4096:
                    assert groups == -(-sm.PERSIST_SLOTS // s) or s == 1
                sch = sm.make_schedule(tile=tile, split_k=s, flags=sm.FLAG_PERSISTENT)
                assert sm.workspace_bytes(sm.MIN_PLUS, sm.DT_I32, n, n, n, sch) == expect, (tile, s, n)
                st, p = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, expect, sch)
                assert st == sm.MM_OK and p["sar_levels"] == s.bit_length() - 1
                assert sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, expect - 1, sch)[0] == sm.MM_ERR_WORKSPACE
    # integer semirings only; no TAR levels, no banding
    sch = sm.make_schedule(split_k=4, flags=sm.FLAG_PERSISTENT)
    assert sm.plan(sm.PLUS_TIMES, sm.DT_F32, 512, 512, 512, 1 << 30, sch)[0] == sm.MM_ERR_UNSUPPORTED
    for bad in (dict(star_depth=1), dict(band_rows=128, tile=128)):
        sch = sm.make_schedule(split_k=4, flags=sm.FLAG_PERSISTENT, **bad)
        assert sm.plan(sm.MIN_PLUS, sm.DT_I32, 512, 512, 512, 1 << 30, sch)[0] == sm.MM_ERR_INVALID_ARG


def test_checked_range_flag_plan_rules():
    chk = sm.FLAG_CHECKED_RANGE
    for sr in (sm.MIN_PLUS, sm.MAX_PLUS, sm.MAX_MIN):
        st, p = sm.plan(sr, sm.DT_I32, 500, 400, 300, 1 << 26, sm.make_schedule(tile=64, split_k=4, flags=chk))
        assert st == sm.MM_OK and p["sched"]["flags"] == chk
        # the same plan as without the flag, apart from the flag
        st2, p2 = sm.plan(sr, sm.DT_I32, 500, 400, 300, 1 << 26, sm.make_schedule(tile=64, split_k=4))
        p2["sched"]["flags"] = chk
        assert p == p2
        st, p = sm.plan(sr, sm.DT_I32, 500, 400, 300, 1 << 26,
                        sm.make_schedule(tile=64, split_k=4, flags=chk | sm.FLAG_PERSISTENT))
        assert st == sm.MM_OK
    for sr, dt in ((sm.OR_AND, sm.DT_I32), (sm.PLUS_TIMES, sm.DT_F32), (sm.PLUS_TIMES, sm.DT_BF16)):
        st, _ = sm.plan(sr, dt, 64, 64, 64, 1 << 26, sm.make_schedule(flags=chk))
        assert st == sm.MM_ERR_INVALID_ARG


def test_domain_violations_rejects_bad_arguments_on_the_host():
    # validation happens before any HIP call, so these need no GPU
    L = _lib.lib()
    cnt = ctypes.c_void_p(16)  # never written: every call below is refused first
    assert L.mm_domain_violations(sm.PLUS_TIMES, 0, None, 0, 0, 1, cnt, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_domain_violations(sm.MIN_PLUS, 0, None, 4, 4, 4, cnt, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_domain_violations(sm.MIN_PLUS, 0, None, 0, 0, 1, None, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_domain_violations(sm.MIN_PLUS, 0, ctypes.c_void_p(16), 4, 8, 4, cnt, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_domain_violations(sm.MIN_PLUS, 0, None, -1, 4, 4, cnt, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_domain_violations(sm.MIN_PLUS, 128, None, 0, 0, 1, cnt, None) == sm.MM_ERR_INVALID_ARG


def test_persistent_status_validates_before_any_hip_call():
    # null workspace or fewer bytes than the control block: refused on the
    # host (no copy, no wait)
    L = _lib.lib()
    assert L.mm_persistent_status(None, 0, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_persistent_status(ctypes.c_void_p(16), 255, None) == sm.MM_ERR_INVALID_ARG
    assert _lib.MM_ERR_INCOMPLETE == -5
    assert L.mm_status_string(sm.MM_ERR_INCOMPLETE).decode().startswith("a bounded wait")


def test_static_scratch_entry_validates_before_any_hip_call():
    # mm_semiring_static checks arguments, flags and the schedule's scratch
    # need on the host, so none of these calls reaches the GPU (none here).
    L = _lib.lib()
    p = ctypes.c_void_p(16)
    assert _lib.STATIC_SCRATCH_BYTES == 64 * MiB
    assert L.mm_semiring_static(1, 0, 4, 4, 4, p, 3, p, 4, p, 4, None, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_semiring_static(1, 0, 4, 4, 4, None, 4, p, 4, p, 4, None, None) == sm.MM_ERR_INVALID_ARG
    assert L.mm_semiring_static(1, 0, 0, 4, 4, None, 4, p, 4, None, 4, None, None) == sm.MM_OK
    pers = sm.make_schedule(tile=64, split_k=2, flags=sm.FLAG_PERSISTENT)
    assert L.mm_semiring_static(1, 0, 64, 64, 64, p, 64, p, 64, p, 64, ctypes.byref(pers), None) == \
        sm.MM_ERR_UNSUPPORTED
    # split 4 over all 4096 rows of an int32 C at once (one band) needs 3
    # temporaries of 64 MiB: refused, and the message names the need and
    # the limit
    big = sm.make_schedule(tile=128, split_k=4, band_rows=4096)
    n = 4096
    assert L.mm_semiring_static(1, 0, n, n, n, p, n, p, n, p, n, ctypes.byref(big), None) == sm.MM_ERR_WORKSPACE
    msg = _lib.last_error()
    assert str(3 * n * n * 4) in msg and str(64 * MiB) in msg
    # left to the planner, the band shrinks until its temporaries fit (the
    # reuse of Sec. sar-mm): 4 bands of 1280 rows
    st, info = sm.plan(sm.MIN_PLUS, sm.DT_I32, n, n, n, 64 * MiB, sm.make_schedule(tile=128, split_k=4))
    assert st == sm.MM_OK and info["bands"] == 4 and info["ws_bytes"] <= 64 * MiB
