"""The schedule space the tuner and the cost model range over: Strassen depth
0-3 x k-split 1, 2, 4, 8 x output tile 32, 64, 128, 256 = 64 schedules (the
256 tile exists for the bf16 kernels only; the planner rejects it for the
int32 semiring kernel, so those entries are infeasible)."""
from __future__ import annotations

import itertools
import math

import paper_1911_05328_amd as sm

DEPTHS = (0, 1, 2, 3)
SPLITS = (1, 2, 4, 8)
TILES = (32, 64, 128, 256)
SCHEDULES = list(itertools.product(DEPTHS, SPLITS, TILES))  # index -> (depth, split, tile)
NSCHED = len(SCHEDULES)
DTYPES = ("f32", "bf16", "i32")  # fp32 via BF16x3 split, bf16 inputs, int32 (min,+)
STRASSEN_VARIANT = sm.WINOGRAD


def supported(dtype: str, depth: int) -> bool:
    """Strassen needs fp32 operands (the split path) and a ring."""
    return depth == 0 or dtype == "f32"


def has_inkernel_variant(dtype: str, idx: int) -> bool:
    """fp32 products without Strassen split their operands into bf16 planes
    when the budget holds them and inside the tile kernel otherwise; both
    variants are timed."""
    return dtype == "f32" and SCHEDULES[idx][0] == 0


def schedule(dtype: str, m: int, idx: int, inkernel: bool = False) -> "sm.Schedule":
    d, s, t = SCHEDULES[idx]
    prec = sm.PREC_BF16X3 if dtype == "f32" else sm.PREC_F32
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
