"""The schedule space the tuner and the cost model range over: Strassen depth
0-3 x k-split 1, 2, 4, 8 x output tile 32, 64, 128, 256 = 64 schedules (the
256 tile exists for the bf16 kernels only; the planner rejects it for the
int32 semiring kernel, so those entries are infeasible).

fp32 products are computed to fp32 accuracy (relative Frobenius error at
most TARGET_ERROR against the float64 product): BF16x3 without Strassen
levels, FP16x3 (22 significant bits per split operand) under Strassen-Winograd
levels, whose pre-additions BF16x3's 16 bits do not absorb (BF16x3 Winograd
levels measured 1.2e-5 to 8.3e-5 at n = 8192, FP16x3 ones 1.9e-6 to
7.0e-6).  The tuner also measures each fp32 schedule's error, and the
proposal leaves out schedules measured above the target."""
from __future__ import annotations

import itertools
import math

import paper_1911_05328_amd as sm

DEPTHS = (0, 1, 2, 3)
SPLITS = (1, 2, 4, 8)
TILES = (32, 64, 128, 256)
SCHEDULES = list(itertools.product(DEPTHS, SPLITS, TILES))  # index -> (depth, split, tile)
NSCHED = len(SCHEDULES)
DTYPES = ("f32", "bf16", "i32")  # fp32 via split precision, bf16 inputs, int32 (min,+)
STRASSEN_VARIANT = sm.WINOGRAD
TARGET_ERROR = 1e-5


def precision(dtype: str, depth: int) -> int:
    """The mm_precision a schedule of the space computes in."""
    if dtype != "f32":
        return sm.PREC_F32
    return sm.PREC_BF16X3 if depth == 0 else sm.PREC_FP16X3


def supported(dtype: str, depth: int) -> bool:
    """Strassen needs fp32 operands (the split path) and a ring."""
    return depth == 0 or dtype == "f32"


def has_inkernel_variant(dtype: str, idx: int) -> bool:
    """fp32 products without Strassen split their operands into bf16 planes
    when the budget holds them and inside the tile kernel otherwise; bf16
    products on 128- and 256-wide tiles copy their operands into planes when
    the budget holds them and stage them straight otherwise; both variants
    are timed."""
    d, _, t = SCHEDULES[idx]
    return (dtype == "f32" and d == 0) or (dtype == "bf16" and t >= 128)


def schedule(dtype: str, m: int, idx: int, inkernel: bool = False) -> "sm.Schedule":
    d, s, t = SCHEDULES[idx]
    prec = precision(dtype, d)
    # non-Strassen schedules run as one band of C, Strassen levels
    # breadth-first (the timed configurations)
    return sm.make_schedule(tile=t, split_k=s, strassen_depth=d, variant=STRASSEN_VARIANT, precision=prec,
                            band_rows=0 if d > 0 else max(m, 1),
                            flags=sm.FLAG_SPLIT_IN_KERNEL if inkernel else 0,
                            strassen_layout=sm.strassen_layout(0) if d > 0 else 0)


def semiring_and_dtype(dtype: str):
    return {"f32": (sm.PLUS_TIMES, sm.DT_F32), "bf16": (sm.PLUS_TIMES, sm.DT_BF16),
            "i32": (sm.MIN_PLUS, sm.DT_I32)}[dtype]


def workspace_bytes(dtype: str, m: int, n: int, k: int, idx: int, inkernel: bool = False):
    """Workspace the schedule needs (None if the combination is unsupported)."""
    if not supported(dtype, SCHEDULES[idx][0]) or (inkernel and not has_inkernel_variant(dtype, idx)):
        return None
    sr, dt = semiring_and_dtype(dtype)
    st, p = sm.plan(sr, dt, m, n, k, 1 << 62, schedule(dtype, m, idx, inkernel))
    return None if st != sm.MM_OK else int(p["ws_bytes"])


def c_elem_bytes(dtype: str) -> int:
    return 4


def features(m: int, n: int, k: int, dtype: str, budget_bytes: float):
    """Inputs of the cost model: log2 sizes, dtype one-hot, log2 of the budget
    relative to the size of C."""
    rel = max(budget_bytes, 1.0) / (m * n * c_elem_bytes(dtype))
    oh = [1.0 if dtype == d else 0.0 for d in DTYPES]
    return [math.log2(m) / 14.0, math.log2(n) / 14.0, math.log2(k) / 14.0, *oh, math.log2(rel) / 3.0]


NFEAT = 7
