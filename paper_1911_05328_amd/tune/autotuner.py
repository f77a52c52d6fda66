"""Exhaustive autotuner: times every supported schedule of the space for a
(shape, dtype) on the GPU, measures each fp32 schedule's error against a
float64 product on sampled rows, and appends one JSON line per shape to a
timing database (resumable: shapes already present are skipped).

Run: python -m paper_1911_05328_amd.tune.autotuner --db PATH [--count 2200]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import space


def shape_list(seed: int, count: int, test_frac: float = 200 / 2200):
    """(m, n, k, dtype, split) rows: m, n, k log-uniform in [128, 16384]
    (int32 (min,+) shapes in [128, 4096], since that kernel is ~30x slower),
    dtype uniform over the three, the last test_frac marked held-out."""
    g = np.random.Generator(np.random.PCG64(seed))
    rows = []
    for i in range(count):
        dtype = space.DTYPES[int(g.integers(0, 3))]
        hi = 4096 if dtype == "i32" else 16384
        m, n, k = (int(round(math.exp(g.uniform(math.log(128), math.log(hi))))) for _ in range(3))
        rows.append((m, n, k, dtype, "test" if i >= count * (1 - test_frac) else "train"))
    return rows


class Timer:
    """Times schedules on the device with buffers reused across shapes."""

    def __init__(self, max_dim: int = 16384):
        import torch
        import paper_1911_05328_amd as sm
        self.torch, self.sm = torch, sm
        dev = torch.device("cuda")
        cap = max_dim * max_dim
        self.fA = torch.randn(cap, device=dev)
        self.fB = torch.randn(cap, device=dev)
        self.fC = torch.zeros(cap, device=dev)
        self.bA = self.fA[: cap // 2].view(torch.bfloat16)
        self.bB = self.fB[: cap // 2].view(torch.bfloat16)
        g = torch.Generator(device=dev).manual_seed(0)
        self.iA = torch.randint(0, 1 << 20, (4096 * 4096,), device=dev, dtype=torch.int32, generator=g)
        self.iB = torch.randint(0, 1 << 20, (4096 * 4096,), device=dev, dtype=torch.int32, generator=g)
        self.iC = torch.full((4096 * 4096,), 1 << 30, device=dev, dtype=torch.int32)
        self.ws = torch.empty(1, dtype=torch.uint8, device=dev)

    def operands(self, dtype, m, n, k):
        if dtype == "f32":
            A, B, C = self.fA, self.fB, self.fC
        elif dtype == "bf16":
            A = self.bA
            B = self.bB
            C = self.fC
        else:
            A, B, C = self.iA, self.iB, self.iC
        return A[: m * k].view(m, k), B[: k * n].view(k, n), C[: m * n].view(m, n)

    def error(self, dtype, m, n, k, idx, rows=16, inkernel=False):
        """Relative Frobenius error of schedule idx's C = A B on `rows` sampled
        output rows against torch's float64 product of the same inputs (fp32
        schedules only; bf16 inputs and (min,+) are exact up to fp32
        accumulation / exact, None)."""
        if dtype != "f32":
            return None
        torch, sm = self.torch, self.sm
        need = space.workspace_bytes(dtype, m, n, k, idx, inkernel)
        if need is None:
            return None
        if need > self.ws.numel():
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        A, B, C = self.operands(dtype, m, n, k)
        C.zero_()
        sm.semiring_mm(A, B, C, sm.PLUS_TIMES, workspace=self.ws[: max(need, 1)] if need else None,
                       schedule=space.schedule(dtype, m, idx, inkernel))
        sel = torch.linspace(0, m - 1, min(rows, m), device="cuda").round().long()
        ref = A[sel].double() @ B.double()
        err = float(torch.linalg.norm(C[sel].double() - ref) / torch.linalg.norm(ref))
        return err

    def time(self, dtype, m, n, k, idx, reps=3, inkernel=False):
        torch, sm = self.torch, self.sm
        need = space.workspace_bytes(dtype, m, n, k, idx, inkernel)
        if need is None:
            return None
        if need > self.ws.numel():
            self.ws = None
            torch.cuda.empty_cache()
            self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        A, B, C = self.operands(dtype, m, n, k)
        sr, _ = space.semiring_and_dtype(dtype)
        sch = space.schedule(dtype, m, idx, inkernel)
        ws = self.ws[: max(need, 1)] if need else None

        def run():
            sm.semiring_mm(A, B, C, sr, workspace=ws, schedule=sch)
        run()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))


def load_db(path):
    rows = []
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                line = line.strip()
                if line:
                    rows.append(json.loads(line))
    return rows


def key(r):
    return (r["m"], r["n"], r["k"], r["dtype"])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", required=True)
    ap.add_argument("--count", type=int, default=2200)
    ap.add_argument("--seed", type=int, default=1911)
    ap.add_argument("--limit-seconds", type=float, default=1e9, help="stop cleanly after this long")
    args = ap.parse_args(argv)
    done = {key(r) for r in load_db(args.db)}
    timer = Timer()
    t_start = time.time()
    todo = [r for r in shape_list(args.seed, args.count) if (r[0], r[1], r[2], r[3]) not in done]
    print(f"{len(done)} shapes in the DB, {len(todo)} to go", flush=True)
    with open(args.db, "a") as f:
        for i, (m, n, k, dtype, split) in enumerate(todo):
            if time.time() - t_start > args.limit_seconds:
                print("time limit reached; resume later", flush=True)
                break
            times = [timer.time(dtype, m, n, k, j) for j in range(space.NSCHED)]
            wsb = [space.workspace_bytes(dtype, m, n, k, j) for j in range(space.NSCHED)]
            # the same schedules splitting inside the tile kernel (no plane space)
            times_ik = [timer.time(dtype, m, n, k, j, inkernel=True) for j in range(space.NSCHED)]
            wsb_ik = [space.workspace_bytes(dtype, m, n, k, j, inkernel=True) for j in range(space.NSCHED)]
            # the error of every timed fp32 schedule (its arithmetic does not
            # depend on the workspace variant: planes and in-kernel split
            # give the same bits)
            errs = [timer.error(dtype, m, n, k, j) if times[j] is not None else None for j in range(space.NSCHED)]
            rec = {"m": m, "n": n, "k": k, "dtype": dtype, "split": split, "times_ms": times, "ws_bytes": wsb,
                   "times_inkernel_ms": times_ik, "ws_inkernel_bytes": wsb_ik, "errors": errs}
            f.write(json.dumps(rec) + "\n")
            f.flush()
            if i % 25 == 0:
                best = min(t for t in times if t is not None)
                print(f"[{i + 1}/{len(todo)}] {dtype} {m}x{n}x{k} best {best:.3f} ms "
                      f"({time.time() - t_start:.0f} s)", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
