"""Seeded random sweep of mm_semiring against the oracle: semiring, dtype,
ragged shape, and a random schedule (tile, k-split, TAR levels (float ones
through the opt-in atomic merge), band,
persistent ring, checked range, Strassen levels and precision) that the
planner accepts under a random workspace budget.  Every case is bit-exact:
integer semirings by definition; (+,x) on small integers, where every
operand, Strassen pre-addition and partial sum is an integer that fp32, bf16
and fp16 hold exactly, so any summation order and split gives the same
bits."""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1911_05328_amd as sm  # noqa: E402
import synth_inputs as si  # noqa: E402

INT_SR = [sm.MIN_PLUS, sm.MAX_PLUS, sm.MAX_MIN, sm.OR_AND]


def draw_case(g):
    kind = g.choice(["int", "int", "f32", "bf16", "f16"])
    m, n, k = (int(x) for x in np.exp(g.uniform(0, np.log(400), 3)).round().clip(1, 400))
    tile = int(g.choice([0, 32, 64, 128, 256]))
    split = int(g.choice([0, 1, 2, 4, 8, 16]))
    sched = dict(tile=tile, split_k=split)
    if kind == "int":
        sr = int(g.choice(INT_SR))
        dt = sm.DT_I32
        if split > 1 and g.random() < 0.3:
            sched["star_depth"] = int(g.integers(0, int(np.log2(split)) + 1))
        if g.random() < 0.2:
            sched["band_rows"] = int(g.choice([32, 64, 128]))
        flags = 0
        if g.random() < 0.25:
            flags |= sm.FLAG_PERSISTENT
            sched.pop("star_depth", None)
            sched.pop("band_rows", None)
        if sr in (sm.MIN_PLUS, sm.MAX_PLUS) and g.random() < 0.4:
            flags |= sm.FLAG_CHECKED_RANGE
        sched["flags"] = flags
    else:
        sr = sm.PLUS_TIMES
        dt = {"f32": sm.DT_F32, "bf16": sm.DT_BF16, "f16": sm.DT_F16}[kind]
        if split > 1 and g.random() < 0.3:
            # TAR levels on floats: atomic merging, opted into (exact here)
            sched["star_depth"] = int(g.integers(1, int(np.log2(split)) + 1))
            sched["flags"] = sm.FLAG_NONDETERMINISTIC
        if kind == "f32":
            p = g.choice(["f32", "bf16x3", "bf16x3", "fp16x3", "strassen"])
            if p == "f32":
                sched["precision"] = sm.PREC_F32
            elif p == "bf16x3":
                sched["precision"] = sm.PREC_BF16X3
                if g.random() < 0.3:
                    sched["flags"] = sched.get("flags", 0) | sm.FLAG_SPLIT_IN_KERNEL
            elif p == "fp16x3":
                sched["precision"] = sm.PREC_FP16X3
                sched.pop("star_depth", None)  # FP16x3 counts star_depth as 8-way levels
                sched.pop("flags", None)
            else:
                sched.pop("flags", None)
                sched.pop("star_depth", None)
                sched["precision"] = int(g.choice([sm.PREC_BF16X3, sm.PREC_BF16X3_HIACC, sm.PREC_FP16X3]))
                sched["strassen_depth"] = int(g.integers(1, 3))
                sched["variant"] = int(g.choice([sm.CLASSIC, sm.WINOGRAD]))
                if g.random() < 0.3:
                    sched["star_depth"] = 1
    budget = int(g.choice([0, 1 << 16, 1 << 20, 1 << 24, 1 << 28]))
    return kind, sr, dt, m, n, k, sched, budget


def operands(g, kind, sr, m, n, k, checked):
    if kind == "int":
        if checked:
            return (si.wide_i32(sr, int(g.integers(1 << 30)), (m, k)), si.wide_i32(sr, int(g.integers(1 << 30)), (k, n)),
                    si.wide_i32(sr, int(g.integers(1 << 30)), (m, n)))
        gen = (lambda s, sh: si.bool_i32(s, sh, 0.05)) if sr == sm.OR_AND else \
            (lambda s, sh: si.semiring_operand(sr, s, sh))
        return gen(int(g.integers(1 << 30)), (m, k)), gen(int(g.integers(1 << 30)), (k, n)), \
            gen(int(g.integers(1 << 30)), (m, n))
    # small integers: |a|, |b| <= 4 keeps Strassen operands (sums of up to 4
    # entries at depth 2, 16 with Winograd growth) and every partial sum
    # (< 400 * 64 * 64) exact in every format
    A = g.integers(-4, 5, (m, k)).astype(np.float32)
    B = g.integers(-4, 5, (k, n)).astype(np.float32)
    C0 = g.integers(-8, 9, (m, n)).astype(np.float32)
    return A, B, C0


def to_dev(x, kind):
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t.to({"bf16": torch.bfloat16, "f16": torch.float16}.get(kind, t.dtype))


def test_random_schedules_bit_exact():
    g = np.random.default_rng(20261202)
    ran = skipped = 0
    while ran < int(os.environ.get("STARMM_SWEEP_CASES", "400")):
        kind, sr, dt, m, n, k, sd, budget = draw_case(g)
        sched = sm.make_schedule(**sd)
        st, p = sm.plan(sr, dt, m, n, k, budget, sched)
        if st != sm.MM_OK:
            skipped += 1
            assert st in (sm.MM_ERR_INVALID_ARG, sm.MM_ERR_UNSUPPORTED, sm.MM_ERR_WORKSPACE)
            continue
        checked = bool(sd.get("flags", 0) & sm.FLAG_CHECKED_RANGE)
        A, B, C0 = operands(g, kind, sr, m, n, k, checked)
        ref = oracle.brute(sr, A.astype(np.int64), B.astype(np.int64), C0.astype(np.int64))
        ws = torch.zeros(max(budget, 1), dtype=torch.uint8, device="cuda") if budget else None
        dC = torch.from_numpy(np.ascontiguousarray(C0)).cuda()
        sm.semiring_mm(to_dev(A, kind), to_dev(B, kind), dC, sr, workspace=ws, schedule=sched)
        torch.cuda.synchronize()
        got = dC.cpu().numpy().astype(np.int64)
        assert np.array_equal(got, ref), (kind, sr, m, n, k, sd, budget, p["sched"])
        ran += 1
    assert skipped < 10 * ran
