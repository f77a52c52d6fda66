#!/usr/bin/env python3
"""Benchmark: effective TFLOP/s (2mnk/t) of the FP32-target Strassen product at
n = 8192 on one MI355X, against the plain 8-way divide-and-conquer fp32 kernel
at the same size, at a relative Frobenius error of at most 1e-5.

One step = one full mm_strassen call (fused pre-additions, the batched
split-precision base products, fused post-additions) on inputs already
resident in HBM.  The (depth, variant, precision) is the fastest candidate
whose error against the oracle's float64 product (all rows) stays within 1e-5
on these inputs; the precisions are BF16x3 and FP16x3 (fp16 hi/lo of operands
scaled per row / column by powers of two).

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "effective TFLOP/s (2mnk/t) vs plain D&C GEMM at equal error; % of MFMA/HBM peak"
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense bf16 MFMA
PEAK_F32_TFLOPS = 157.3     # MI355X dense fp32 MFMA
PEAK_HBM_GBS = 8000.0
TARGET_ERR = 1e-5
N = 8192
# precision codes of the library (mm_precision)
PREC_BF16X3_CODE, PREC_FP16X3_CODE = 1, 4
PREC_NAME = {PREC_BF16X3_CODE: "bf16x3", PREC_FP16X3_CODE: "fp16x3"}
PREC_DESC = {PREC_BF16X3_CODE: "BF16x3 split, fp32 accumulate",
             PREC_FP16X3_CODE: "FP16x3 split of power-of-two row/column-scaled operands, fp32 accumulate"}
KERNEL_NAME = {PREC_BF16X3_CODE: "bf16x3_tile", PREC_FP16X3_CODE: "fp16x3_tile"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def sampled_err(C, A64rows, B64, rows, torch):
    ref = A64rows @ B64
    got = C[rows].double()
    return float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))


class OracleReference:
    """Part of the cpu_baseline leg: the oracle's float64 classical product
    (O-5) of a whole input pair, computed on the host once per input set and
    outside every timed region; the errors this benchmark reports are taken
    against it on all rows (relative Frobenius, and for the chosen
    configuration the componentwise and per-row errors as well)."""

    def __init__(self):
        import oracle
        self.oracle = oracle
        self.refs = {}
        self.seconds = {}

    def ref(self, name, A_np, B_np):
        if name not in self.refs:
            t0 = time.perf_counter()
            self.refs[name] = (self.oracle.fp64_ref(A_np, B_np), A_np, B_np)
            self.seconds[name] = time.perf_counter() - t0
            log(f"oracle reference {name}: {self.seconds[name]:.1f} s")
        return self.refs[name][0]

    def drop(self, name):
        self.refs.pop(name, None)

    def rel_fro(self, name, C):
        return self.oracle.rel_fro(C.cpu().numpy(), self.refs[name][0])

    def detail(self, name, C):
        import numpy as np
        R, A_np, B_np = self.refs[name]
        Ch = C.cpu().numpy()
        rows = self.oracle.row_rel_err(Ch, R)
        return {"rel_fro_err": self.oracle.rel_fro(Ch, R),
                "componentwise_max": self.oracle.componentwise_err(Ch, R, A_np, B_np),
                "row_rel_err_max": float(rows.max()), "row_rel_err_median": float(np.median(rows)),
                "rows_over_target": int((rows > TARGET_ERR).sum())}


# Sources of the base-product tile kernels (the traffic figure is valid only
# for the code it was measured on).
TILE_SOURCES = ["paper_1911_05328_amd/csrc/k_gemm_bf16.hip", "paper_1911_05328_amd/csrc/tile_bf16.hpp",
                "paper_1911_05328_amd/csrc/tile_dma.hpp"]


def sources_sha256(paths):
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()


def kernel_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the kernel sources as they are now; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    srcs = d.get("sources", [])
    if not srcs or not all(os.path.exists(os.path.join(ROOT, s)) for s in srcs):
        return None
    if sources_sha256(srcs) != d.get("sources_sha256"):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(depth: int, variant: int):
    """The oracle's Strassen (float64, same depth and variant) on a bounded
    sub-problem of the workload, timed on the host cores."""
    import numpy as np

    import oracle
    import synth_inputs as si
    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    n_s, t = 512, 0.0
    while True:
        A = si.normal_f32(si.BASE_SEED, (n_s, n_s)).astype(np.float64)
        B = si.normal_f32(si.BASE_SEED + 1, (n_s, n_s)).astype(np.float64)
        t0 = time.perf_counter()
        oracle.strassen(A, B, depth, variant)
        t = time.perf_counter() - t0
        # the next doubling costs ~7-8x; stop once it would exceed ~25 s
        if n_s >= N or t * 8 > 25.0:
            break
        n_s *= 2
    # the same on one core, on 1/64 of the work (a quarter of the size)
    n1 = max(n_s // 4, 256)
    A = si.normal_f32(si.BASE_SEED, (n1, n1)).astype(np.float64)
    B = si.normal_f32(si.BASE_SEED + 1, (n1, n1)).astype(np.float64)
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.strassen(A, B, depth, variant)
    t1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    # the plain 8-way recursion at n = 256, base 32 (float64), for the small
    # configuration's comparison entry
    A = si.uniform_f32(si.BASE_SEED, (256, 256)).astype(np.float64)
    B = si.uniform_f32(si.BASE_SEED + 1, (256, 256)).astype(np.float64)
    t0 = time.perf_counter()
    oracle.rec8(oracle.PLUS_TIMES, A, B, b=32)
    t_small = time.perf_counter() - t0
    return {"value": 2.0 * n_s ** 3 / t / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "plain_dc_n256_ms": t_small * 1e3,
            "sample": f"oracle float64 Strassen ({'Winograd' if variant else 'classic'}, depth {depth}) on one "
                      f"n={n_s} square product of the same N(0,1) recipe, {t:.2f} s wall",
            "one_core": {"value": 2.0 * n1 ** 3 / t1 / 1e12, "unit": "TFLOP/s", "cores": 1,
                         "sample": f"the same at n={n1}, {t1:.2f} s wall"}}


def digest_rocprof(stats_db: str, fetch_db: str, write_db: str, depth: int, variant: int, prec: int,
                   command: str) -> None:
    """Write the committed summaries under profiles/ from rocprofv3 outputs:
    the kernel-trace statistics of a bench run, and HBM traffic per launch of
    the base-product kernel from FETCH_SIZE / WRITE_SIZE runs, each scaled by
    what the counter reads for a 512 MiB device copy."""
    import sqlite3
    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    c = sqlite3.connect(stats_db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    lines = [f"# Kernel time, Strassen FP32-target n={N} bench run", "",
             f"Command: `{command}`", "",
             "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in rows[:16]:
        short = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0][:90]
        lines.append(f"| `{short}` | {calls} | {tot:.1f} | {avg:.1f} | {pct:.1f} |")
    # the tile kernel per launch grid: the bench also times other depths, so
    # the chosen depth's launches are told apart by their grid
    leaf = -(-N // 2 ** depth)
    chosen_grid = (-(-leaf // 256)) ** 2 * 7 ** depth * 512
    lines += ["", "Base-product tile kernel by launch grid (threads):", "",
              "| kernel | grid threads | calls | average us | chosen depth |", "|---|---|---|---|---|"]
    for name, grid, calls, avg in c.execute(
            "select name, grid_x, count(*), avg(duration) / 1000.0 from kernels "
            "where name like '%k_bf16x3_dma%' group by name, grid_x order by name, grid_x"):
        short = name.replace("(anonymous namespace)::", "").split("(")[0]
        chosen = grid == chosen_grid and ("<true>" in short) == (prec == PREC_FP16X3_CODE)
        lines.append(f"| `{short}` | {grid} | {calls} | {avg:.1f} | {'yes' if chosen else ''} |")
    open(os.path.join(prof, f"kernels_strassen_n{N}.md"), "w").write("\n".join(lines) + "\n")

    def per_dispatch(db, counter):
        cc = sqlite3.connect(db)
        out = {}
        for name, val in cc.execute("select kernel_name, value from counters_collection where counter_name=?",
                                    (counter,)):
            out.setdefault(name, []).append(float(val))
        return out
    fetch, write = per_dispatch(fetch_db, "FETCH_SIZE"), per_dispatch(write_db, "WRITE_SIZE")
    copy_kib = 512 * 1024.0

    def pick(d, key):
        vals = [v for k, vs in d.items() if key in k for v in vs]
        return sum(vals) / len(vals) if vals else None
    f_copy, w_copy = pick(fetch, "copyBuffer"), pick(write, "copyBuffer")
    f_scale, w_scale = copy_kib / f_copy, copy_kib / w_copy
    # the wide planes tile (direct-to-LDS copies) runs the n = 8192 leaves
    key = "k_bf16x3_dma" if any("k_bf16x3_dma" in k for k in fetch) else "k_bf16_tile"
    f_k, w_k = pick(fetch, key), pick(write, key)
    hbm = (f_k * f_scale + w_k * w_scale) * 1024.0
    leaf = -(-N // 2 ** depth)
    algo = 7 ** depth * (2 * leaf * leaf * 4 + leaf * leaf * 4)
    rec = {"kernel": KERNEL_NAME[prec], "device_kernel": key, "workload": f"strassen_n{N}_d{depth}",
           "variant": "winograd" if variant else "classic", "sources": TILE_SOURCES,
           "sources_sha256": sources_sha256(TILE_SOURCES),
           "fetch_kib_raw": f_k, "write_kib_raw": w_k, "copy_fetch_kib_raw": f_copy,
           "copy_write_kib_raw": w_copy, "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": algo,
           "command_fetch": f"rocprofv3 --pmc FETCH_SIZE -d <out>/pmc_fetch -o fetch -- python3 bench.py "
                            f"--profile-only {depth} {variant} {prec}",
           "command_write": f"rocprofv3 --pmc WRITE_SIZE -d <out>/pmc_write -o write -- python3 bench.py "
                            f"--profile-only {depth} {variant} {prec}"}
    json.dump(rec, open(os.path.join(prof, f"traffic_{KERNEL_NAME[prec]}_strassen_n{N}_d{depth}.json"), "w"),
              indent=1)
    print(json.dumps(rec, indent=1))


def batched_inputs(si, torch, dev):
    """The 512 uneven bf16 products: shapes log-uniform in [64, 4096],
    N(0,1) operands from torch's seeded generator, fp32 C zeros."""
    shapes = [tuple(int(v) for v in r) for r in si.batched_shapes(si.BASE_SEED, 512)]
    gen = torch.Generator(device=dev).manual_seed(si.BASE_SEED)
    trip = [(torch.randn(m, k, device=dev, generator=gen).to(torch.bfloat16),
             torch.randn(k, n, device=dev, generator=gen).to(torch.bfloat16),
             torch.zeros(m, n, device=dev)) for m, n, k in shapes]
    return shapes, trip


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", nargs=3, type=int, metavar=("DEPTH", "VARIANT", "PRECISION"),
                    help="run only a 512 MiB copy (counter calibration) and 3 Strassen steps, for rocprofv3")
    ap.add_argument("--profile-batched", type=int, metavar="LAUNCHES",
                    help="run only the 512-problem batched graph LAUNCHES times, for rocprofv3")
    ap.add_argument("--profile-minplus", type=int, metavar="LAUNCHES",
                    help="run only the (min,+) n=4096 unsplit product LAUNCHES times, for rocprofv3")
    ap.add_argument("--profile-bf16", type=int, metavar="LAUNCHES",
                    help="run only a 512 MiB copy (counter calibration) and the one-plane bf16 8192^3 product "
                         "LAUNCHES times, for rocprofv3")
    ap.add_argument("--profile-valu", type=int, metavar="LAUNCHES",
                    help="run only the register-only int32 VALU microbenchmark, then the (min,+) n=4096 "
                         "unsplit product, LAUNCHES times each, for rocprofv3 counters")
    ap.add_argument("--digest-rocprof", nargs=6,
                    metavar=("STATS_DB", "FETCH_DB", "WRITE_DB", "DEPTH", "VARIANT", "PRECISION"),
                    help="write profiles/ summaries from rocprofv3 databases (no GPU needed)")
    args = ap.parse_args()
    if args.digest_rocprof:
        s_db, f_db, w_db, d, v, p = args.digest_rocprof
        digest_rocprof(s_db, f_db, w_db, int(d), int(v), int(p),
                       "rocprofv3 --kernel-trace --stats -d <out>/prof_bench -o bench -- "
                       "python3 bench.py --steps 5 --warmup 2 --no-cpu-baseline")
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1911_05328_amd as sm
    import synth_inputs as si

    dev = torch.device("cuda:0")
    if args.profile_only:
        d, v, p = args.profile_only
        A = torch.from_numpy(si.normal_f32(si.BASE_SEED, (N, N))).to(dev)
        B = torch.from_numpy(si.normal_f32(si.BASE_SEED + 1, (N, N))).to(dev)
        C = torch.zeros((N, N), dtype=torch.float32, device=dev)
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        ws = torch.empty(max(sm.strassen_workspace_bytes(N, N, N, d, v, p), 1),
                         dtype=torch.uint8, device=dev)
        for _ in range(3):
            sm.strassen_mm(A, B, C, d, v, p, workspace=ws)
        torch.cuda.synchronize()
        log("profile-only done")
        return 0
    if args.profile_bf16:
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        gen = torch.Generator(device=dev).manual_seed(si.BASE_SEED)
        Ab = torch.randn(N, N, device=dev, generator=gen).to(torch.bfloat16)
        Bb = torch.randn(N, N, device=dev, generator=gen).to(torch.bfloat16)
        Cb = torch.zeros((N, N), device=dev)
        sch = sm.make_schedule(tile=256, split_k=1)
        wsb = torch.empty(sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_BF16, N, N, N, sch), dtype=torch.uint8, device=dev)
        for _ in range(args.profile_bf16):
            sm.semiring_mm(Ab, Bb, Cb, sm.PLUS_TIMES, workspace=wsb, schedule=sch)
        torch.cuda.synchronize()
        log("profile-bf16 done")
        return 0
    if args.profile_valu:
        import ctypes
        from paper_1911_05328_amd import _lib
        small = torch.empty(1 << 16, dtype=torch.int32, device=dev)
        work = ctypes.c_double()
        for _ in range(args.profile_valu):
            st = _lib.lib().mm_microbench(0, 20000, ctypes.c_void_p(small.data_ptr()), None, 0, ctypes.byref(work),
                                          None)
            if st != sm.MM_OK:
                raise sm.StarmmError(st, "mm_microbench")
        torch.cuda.synchronize()
        args.profile_minplus = args.profile_valu
    if args.profile_minplus:
        n2 = 4096
        Ai = torch.from_numpy(si.minplus_i32(si.BASE_SEED, (n2, n2))).to(dev)
        Bi = torch.from_numpy(si.minplus_i32(si.BASE_SEED + 1, (n2, n2))).to(dev)
        Ci = torch.full((n2, n2), sm.INF, dtype=torch.int32, device=dev)
        for _ in range(args.profile_minplus):
            sm.semiring_mm(Ai, Bi, Ci, sm.MIN_PLUS, schedule=sm.make_schedule(tile=128, split_k=1))
        torch.cuda.synchronize()
        log("profile-minplus done")
        return 0
    if args.profile_batched:
        _, trip = batched_inputs(si, torch, dev)
        wsb = torch.empty(sm.batched_workspace_bytes(trip), dtype=torch.uint8, device=dev)
        graph = sm.BatchedGraph(trip, workspace=wsb)
        for _ in range(args.profile_batched):
            graph.launch()
        torch.cuda.synchronize()
        graph.close()
        log("profile-batched done")
        return 0
    log("generating inputs")
    A_np = si.normal_f32(si.BASE_SEED, (N, N))
    B_np = si.normal_f32(si.BASE_SEED + 1, (N, N))
    A = torch.from_numpy(A_np).to(dev)
    B = torch.from_numpy(B_np).to(dev)
    C = torch.zeros((N, N), dtype=torch.float32, device=dev)
    rows = torch.from_numpy(np.unique(np.random.default_rng(7).integers(0, N, 48))).to(dev)
    A64rows = A[rows].double()
    B64 = B.double()
    # errors: against the oracle's float64 product on all rows (the
    # cpu_baseline leg), or without that leg against torch's float64 product
    # on 48 sampled rows
    oref = None
    if not args.no_cpu_baseline:
        oref = OracleReference()
        oref.ref("normal", A_np, B_np)

    def err_of(C, name="normal", A64r=None, B64r=None):
        if oref is not None:
            return oref.rel_fro(name, C)
        return sampled_err(C, A64rows if A64r is None else A64r, B64 if B64r is None else B64r, rows, torch)
    err_kind = "oracle float64 product, all rows" if oref is not None else "torch float64 product, 48 sampled rows"

    # ---- the plain 8-way D&C fp32 kernel: the comparison point
    plain = sm.make_schedule(tile=128, split_k=1, precision=sm.PREC_F32)

    def run_plain():
        sm.semiring_mm(A, B, C, sm.PLUS_TIMES, schedule=plain)

    C.zero_()
    run_plain()
    torch.cuda.synchronize()
    err_plain = err_of(C)
    ms_plain = timed_steps(run_plain, max(3, args.steps // 2), 2, torch)
    tf_plain = 2.0 * N ** 3 / (ms_plain * 1e-3) / 1e12
    log(f"plain D&C fp32: {ms_plain:.3f} ms, {tf_plain:.1f} TFLOP/s, err {err_plain:.2e}")

    # the small plain case: n = 256, base tile 32, A, B ~ U[-1, 1] (one
    # launch, latency-bound: 3.4e7 flop take 0.2 us at the fp32 MFMA peak)
    n1 = 256
    A1 = torch.from_numpy(si.uniform_f32(si.BASE_SEED, (n1, n1))).to(dev)
    B1 = torch.from_numpy(si.uniform_f32(si.BASE_SEED + 1, (n1, n1))).to(dev)
    C1 = torch.zeros((n1, n1), dtype=torch.float32, device=dev)
    small = sm.make_schedule(tile=32, split_k=1, precision=sm.PREC_F32)
    C1.zero_()
    sm.semiring_mm(A1, B1, C1, sm.PLUS_TIMES, schedule=small)
    torch.cuda.synchronize()
    ref1 = A1.double() @ B1.double()
    err_small = float((C1.double() - ref1).norm() / ref1.norm())
    ms_small = timed_steps(lambda: sm.semiring_mm(A1, B1, C1, sm.PLUS_TIMES, schedule=small), 50, 5, torch)
    del A1, B1, C1, ref1

    # ---- candidate Strassen configurations (depth 1-3, the workload's
    # range); keep those within the error target.  The split-precision
    # product without Strassen levels (depth 0) is timed beside them as a
    # comparison, not a candidate.
    cands = [(d, v, p) for p in (sm.PREC_BF16X3, sm.PREC_FP16X3)
             for d, v in ((1, sm.CLASSIC), (1, sm.WINOGRAD), (2, sm.CLASSIC), (2, sm.WINOGRAD),
                          (3, sm.CLASSIC), (3, sm.WINOGRAD))]
    depth0 = [(0, sm.WINOGRAD, sm.PREC_BF16X3), (0, sm.WINOGRAD, sm.PREC_FP16X3)]
    ws_bytes = max(sm.strassen_workspace_bytes(N, N, N, d, v, p) for d, v, p in cands + depth0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    results, depth0_results = [], {}
    for d, v, p in cands + depth0:
        def run(d=d, v=v, p=p):
            sm.strassen_mm(A, B, C, d, v, p, workspace=ws)
        C.zero_()
        run()
        torch.cuda.synchronize()
        err = err_of(C)
        ms = timed_steps(run, 10, 5, torch)
        if d == 0:
            depth0_results[PREC_NAME[p]] = {"ms": ms, "tflops_effective": 2.0 * N ** 3 / (ms * 1e-3) / 1e12,
                                            "rel_fro_err": err}
        else:
            results.append((d, v, p, err, ms))
        log(f"candidate {PREC_NAME[p]} depth={d} variant={'W' if v else 'C'}: {ms:.3f} ms, err {err:.2e}")
    ok = [r for r in results if r[3] <= TARGET_ERR]
    depth, variant, prec, _, _ = min(ok, key=lambda r: r[4]) if ok else min(results, key=lambda r: r[3])

    def step():
        sm.strassen_mm(A, B, C, depth, variant, prec, workspace=ws)

    C.zero_()
    step()
    torch.cuda.synchronize()
    err = err_of(C)
    err_detail = oref.detail("normal", C) if oref is not None else None

    # ---- timed region: exactly K steps, profiler events on the launch stream
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sm.profile_reset()
    sm.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    sm.profile_enable(False)
    prof = sm.profile_summary()
    sm.profile_reset()
    value = 2.0 * N ** 3 / (ms * 1e-3) / 1e12

    # per-step spread, after the timed region: 20 steps each bracketed by HIP
    # events on the launch stream (median, p10, p90)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for e0, e1 in evs:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    per_step = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    step_stats = {"median_ms": float(np.median(per_step)), "p10_ms": float(np.percentile(per_step, 10)),
                  "p90_ms": float(np.percentile(per_step, 90)), "steps": len(evs)}

    # the same step captured once in a HIP graph and replayed (a call only
    # enqueues kernels): what the gaps between its launches cost
    graph_step = None
    try:
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            step()
        for _ in range(3):
            graph.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        for _ in range(20):
            graph.replay()
        g1.record()
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1) / 20
        graph_step = {"ms": gms, "tflops_effective": 2.0 * N ** 3 / (gms * 1e-3) / 1e12,
                      "eager_step_median_ms": step_stats["median_ms"], "replays": 20}
        del graph
    except Exception as e:
        graph_step = {"error": repr(e)}

    kname = KERNEL_NAME[prec]
    launches, kms = prof.get(kname, (0, 0.0))
    leaf = -(-N // 2 ** depth)
    flops_per_launch = 3 * 2.0 * leaf ** 3 * 7 ** depth
    achieved = flops_per_launch / (kms / max(launches, 1) * 1e-3) / 1e12 if launches else None
    roofline = {"bound": "mfma", "kernel": kname, "achieved": achieved, "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": (achieved / PEAK_BF16_TFLOPS) if achieved else None,
                "traffic": kernel_traffic(kname, f"strassen_n{N}_d{depth}"),
                "avg_launch_ms": kms / max(launches, 1) if launches else None,
                "flops_per_launch": flops_per_launch,
                "kernel_ms_per_step": {k: v[1] / args.steps for k, v in prof.items()}}
    # the HBM-bound addition passes beside the tile: algorithmic bytes per
    # step (4 B per element read or written, hi + lo planes 4 B together)
    g7 = (7.0 / 4.0) ** depth
    for kname2, nbytes in (("strassen_pre", 2 * (1.0 + g7) * N * N * 4), ("strassen_post", (g7 + 2.0) * N * N * 4)):
        if kname2 in prof:
            kms2 = prof[kname2][1] / args.steps
            roofline.setdefault("hbm_passes", {})[kname2] = {
                "bytes_per_step": nbytes, "ms_per_step": kms2,
                "frac_of_8TBs": nbytes / (kms2 * 1e-3) / (PEAK_HBM_GBS * 1e9)}

    # ---- the chosen levels on the second input set (rows of A and B scaled
    # by 10^U(-3,3)) and with the fp64 pre/post additions
    sets = {}
    try:
        As_np = si.row_scaled_normal_f32(si.BASE_SEED, (N, N))
        Bs_np = si.row_scaled_normal_f32(si.BASE_SEED + 1, (N, N))
        As = torch.from_numpy(As_np).to(dev)
        Bs = torch.from_numpy(Bs_np).to(dev)
        As64rows, Bs64 = As[rows].double(), Bs.double()
        hiacc = {sm.PREC_BF16X3: sm.PREC_BF16X3_HIACC, sm.PREC_FP16X3: sm.PREC_FP16X3_HIACC}[prec]
        for dname, (AA, BB, A64r, B64r, An, Bn) in (("normal", (A, B, A64rows, B64, A_np, B_np)),
                                                    ("rows_scaled", (As, Bs, As64rows, Bs64, As_np, Bs_np)),
                                                    ("a_rows_scaled", (As, B, As64rows, B64, As_np, B_np))):
            if oref is not None:
                oref.ref(dname, An, Bn)
            for label, p_ in (("chosen", prec), ("fp64_additions", hiacc)):
                def run_set(AA=AA, BB=BB, p_=p_):
                    sm.strassen_mm(AA, BB, C, depth, variant, p_, workspace=ws)
                C.zero_()
                run_set()
                torch.cuda.synchronize()
                ent = sets.setdefault(label, {})
                ent[dname] = oref.detail(dname, C) if oref is not None else \
                    {"rel_fro_err": sampled_err(C, A64r, B64r, rows, torch)}
                if dname == "normal":
                    ent[dname]["ms"] = timed_steps(run_set, 5, 1, torch)
            if oref is not None and dname != "normal":
                oref.drop(dname)
        del As, Bs, As64rows, Bs64, As_np, Bs_np
        sets["error_reference"] = err_kind
    except Exception as e:
        sets["error"] = repr(e)

    # ---- space-time trade: STAR-Strassen (t 8-way levels above the chosen
    # Strassen levels) at the same n, workspace vs time
    star = {}
    try:
        full_ws = sm.strassen_workspace_bytes(N, N, N, depth, variant, prec)
        star["t0"] = {"ms": ms, "workspace_bytes": full_ws}
        for t in (1, 2):
            sch = sm.make_schedule(strassen_depth=depth, star_depth=t, variant=variant, precision=prec)
            need = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, N, N, N, sch)

            def run_star(sch=sch, need=need):
                sm.semiring_mm(A, B, C, sm.PLUS_TIMES, workspace=ws[:need], schedule=sch)
            mst = timed_steps(run_star, max(3, args.steps // 2), 2, torch)
            star[f"t{t}"] = {"ms": mst, "workspace_bytes": need, "tflops": 2.0 * N ** 3 / (mst * 1e-3) / 1e12}
    except Exception as e:
        star["error"] = repr(e)

    # ---- space-time trade inside the Strassen levels: t of them depth-first
    # on top (SAR-Strassen: 7^t rounds, each forming only its own leaves and
    # adding its product into C at once) over breadth-first ones
    layouts = {}
    try:
        for d_, t_ in ((1, 0), (1, 1), (2, 0), (2, 1), (2, 2)):
            sch = sm.make_schedule(strassen_depth=d_, variant=sm.CLASSIC, precision=sm.PREC_BF16X3,
                                   strassen_layout=sm.strassen_layout((1 << t_) - 1))
            need = sm.workspace_bytes(sm.PLUS_TIMES, sm.DT_F32, N, N, N, sch)
            wsl = ws[:need] if need <= ws.numel() else torch.empty(need, dtype=torch.uint8, device=dev)

            def run_layout(sch=sch, wsl=wsl):
                sm.semiring_mm(A, B, C, sm.PLUS_TIMES, workspace=wsl, schedule=sch)
            C.zero_()
            run_layout()
            torch.cuda.synchronize()
            errl = err_of(C)
            msl = timed_steps(run_layout, max(3, args.steps // 2), 2, torch)
            layouts[f"d{d_}_t{t_}"] = {"depth": d_, "depth_first_levels": t_, "ms": msl,
                                       "tflops_effective": 2.0 * N ** 3 / (msl * 1e-3) / 1e12,
                                       "workspace_bytes": need, "rel_fro_err": errl}
            del wsl
        layouts["variant"] = "classic, BF16x3"
    except Exception as e:
        layouts["error"] = repr(e)

    # ---- general bilinear level (eq. bilinear): the same n = 8192 product
    # through one level of a scheme given as coefficients
    bilinear = {}
    try:
        st_c = sm.bilinear_scheme(sm.BILINEAR_STRASSEN, sm.CLASSIC)
        for label, scheme in (("strassen_g2_r7", st_c), ("classical_g2_r8", sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, 2)),
                              ("strassen_x_strassen_g4_r49", sm.bilinear_scheme_product(st_c, st_c)),
                              ("classical_g4_r64", sm.bilinear_scheme(sm.BILINEAR_CLASSICAL, 4))):
            need = sm.bilinear_workspace_bytes(N, N, N, scheme)
            wsb = ws[:need] if need <= ws.numel() else torch.empty(need, dtype=torch.uint8, device=dev)

            def run_bilinear(scheme=scheme, wsb=wsb):
                sm.bilinear_mm(A, B, C, scheme, workspace=wsb)
            C.zero_()
            run_bilinear()
            torch.cuda.synchronize()
            errb = err_of(C)
            msb = timed_steps(run_bilinear, max(3, args.steps // 2), 2, torch)
            bilinear[label] = {"grid": scheme.g, "products": scheme.products, "ms": msb,
                               "tflops_effective": 2.0 * N ** 3 / (msb * 1e-3) / 1e12, "workspace_bytes": need,
                               "rel_fro_err": errb}
            del wsb
        bilinear["precision"] = "BF16x3 base product, fp32 additions"
    except Exception as e:
        bilinear["error"] = repr(e)

    # ---- (min,+) int32 n = 4096: the exact-semiring path, plain and split
    secondary = {}
    try:
        n2 = 4096
        Ai = torch.from_numpy(si.minplus_i32(si.BASE_SEED, (n2, n2))).to(dev)
        Bi = torch.from_numpy(si.minplus_i32(si.BASE_SEED + 1, (n2, n2))).to(dev)
        Ci = torch.full((n2, n2), sm.INF, dtype=torch.int32, device=dev)
        wsi = torch.empty(4 * n2 * n2 * 4, dtype=torch.uint8, device=dev)
        C_plain = None
        for label, sch, wsx in (("plain_s1", sm.make_schedule(tile=128, split_k=1), 0),
                                ("budget_1x_s2", sm.make_schedule(tile=128, split_k=2), 1),
                                ("budget_2x_s2", sm.make_schedule(tile=128, split_k=2), 2),
                                ("budget_4x_s4", sm.make_schedule(tile=128, split_k=4), 4),
                                ("tar_s4", sm.make_schedule(tile=128, split_k=4, star_depth=2), 0),
                                ("persistent_s4", sm.make_schedule(tile=128, split_k=4, flags=sm.FLAG_PERSISTENT), -1)):
            if wsx < 0:  # the persistent slot ring: a fixed size, whatever n is
                wv = wsi[: sm.workspace_bytes(sm.MIN_PLUS, sm.DT_I32, n2, n2, n2, sch)]
            else:
                wv = wsi[: wsx * n2 * n2 * 4] if wsx else None

            def mp(sch=sch, wv=wv):
                sm.semiring_mm(Ai, Bi, Ci, sm.MIN_PLUS, workspace=wv, schedule=sch, check_persistent=False)
            # one product from C = INF, compared in full with the unsplit
            # schedule's (which every exact schedule must reproduce bit for bit)
            Ci.fill_(sm.INF)
            mp()
            if sch.flags & sm.FLAG_PERSISTENT:
                sm.persistent_status(wv)  # raises if a bounded wait gave up
            torch.cuda.synchronize()
            if C_plain is None:
                C_plain = Ci.clone()
            same = bool(torch.equal(Ci, C_plain))
            msi = timed_steps(mp, max(3, args.steps // 2), 2, torch)
            if sch.flags & sm.FLAG_PERSISTENT:
                sm.persistent_status(wv)
            secondary[label] = {"ms": msi, "Tops_effective": 2.0 * n2 ** 3 / (msi * 1e-3) / 1e12,
                                "valu_Tops": 1.5 * n2 ** 3 / (msi * 1e-3) / 1e12,
                                "workspace_bytes": 0 if wv is None else wv.numel(),
                                "equal_to_plain_s1": same}
        # entries of either sign (negative weights) through the checked range
        Aw = torch.from_numpy(si.wide_i32(sm.MIN_PLUS, si.BASE_SEED, (n2, n2))).to(dev)
        Bw = torch.from_numpy(si.wide_i32(sm.MIN_PLUS, si.BASE_SEED + 1, (n2, n2))).to(dev)
        for label, sch, wsx in (("checked_wide_s1", sm.make_schedule(tile=128, split_k=1, flags=sm.FLAG_CHECKED_RANGE), 0),
                                ("checked_wide_budget_4x_s4",
                                 sm.make_schedule(tile=128, split_k=4, flags=sm.FLAG_CHECKED_RANGE), 4)):
            wv = wsi[: wsx * n2 * n2 * 4] if wsx else None

            def mpw(sch=sch, wv=wv):
                sm.semiring_mm(Aw, Bw, Ci, sm.MIN_PLUS, workspace=wv, schedule=sch)
            msi = timed_steps(mpw, max(3, args.steps // 2), 2, torch)
            secondary[label] = {"ms": msi, "Tops_effective": 2.0 * n2 ** 3 / (msi * 1e-3) / 1e12,
                                "valu_Tops": 1.5 * n2 ** 3 / (msi * 1e-3) / 1e12,
                                "workspace_bytes": 0 if wv is None else wv.numel()}
        del Ai, Bi, Ci, Aw, Bw, C_plain
        # few tiles, deep k (m = n = 1024, k = 16384: 64 tiles of 128 for
        # 256 CUs): the k-split is what fills the GPU, and its temporaries
        # are what the workspace budget pays for (Sec. sar-mm, Sec. tar-mm)
        md, kd = 1024, 16384
        Ad = torch.from_numpy(si.minplus_i32(si.BASE_SEED + 2, (md, kd))).to(dev)
        Bd = torch.from_numpy(si.minplus_i32(si.BASE_SEED + 3, (kd, md))).to(dev)
        Cd = torch.full((md, md), sm.INF, dtype=torch.int32, device=dev)
        deep = {}
        for label, sch in (("s1", sm.make_schedule(tile=128, split_k=1)),
                           ("s4_temps", sm.make_schedule(tile=128, split_k=4)),
                           ("s16_temps", sm.make_schedule(tile=128, split_k=16)),
                           ("s16_tar", sm.make_schedule(tile=128, split_k=16, star_depth=4)),
                           ("s16_star2", sm.make_schedule(tile=128, split_k=16, star_depth=2)),
                           ("s16_persistent", sm.make_schedule(tile=128, split_k=16, flags=sm.FLAG_PERSISTENT))):
            need = sm.workspace_bytes(sm.MIN_PLUS, sm.DT_I32, md, md, kd, sch)
            wv = wsi[:need] if need else None

            def opd(sch=sch, wv=wv):
                sm.semiring_mm(Ad, Bd, Cd, sm.MIN_PLUS, workspace=wv, schedule=sch, check_persistent=False)
            msd = timed_steps(opd, max(3, args.steps // 5), 2, torch)
            if sch.flags & sm.FLAG_PERSISTENT:
                sm.persistent_status(wv)
            deep[label] = {"ms": msd, "Tops_effective": 2.0 * md * md * kd / (msd * 1e-3) / 1e12,
                           "workspace_bytes": need}
        secondary["deep_k_1024x1024x16384"] = deep
        del Ad, Bd, Cd, wsi
        # the other exact semirings on the same VALU kernel, plain schedule
        for label, sr, gen, init in (("maxmin_s1", sm.MAX_MIN, si.maxmin_i32, si.I32_MIN),
                                     ("bool_s1", sm.OR_AND, lambda s, sh: si.bool_i32(s, sh, 1.0 / 64), 0)):
            Ai = torch.from_numpy(gen(si.BASE_SEED, (n2, n2))).to(dev)
            Bi = torch.from_numpy(gen(si.BASE_SEED + 1, (n2, n2))).to(dev)
            Ci = torch.full((n2, n2), init, dtype=torch.int32, device=dev)

            def op(sr=sr, Ai=Ai, Bi=Bi, Ci=Ci):
                sm.semiring_mm(Ai, Bi, Ci, sr, schedule=sm.make_schedule(tile=128, split_k=1))
            msi = timed_steps(op, max(3, args.steps // 2), 2, torch)
            secondary[label] = {"ms": msi, "Tops_effective": 2.0 * n2 ** 3 / (msi * 1e-3) / 1e12}
            del Ai, Bi, Ci
    except Exception as e:  # the headline stands on its own
        secondary["error"] = repr(e)

    # ---- 512 uneven bf16 products in one persistent graph-captured launch
    batched = {}
    try:
        shapes, trip = batched_inputs(si, torch, dev)
        wsb = torch.empty(sm.batched_workspace_bytes(trip), dtype=torch.uint8, device=dev)
        graph = sm.BatchedGraph(trip, workspace=wsb)
        for _, _, Cb in trip:
            Cb.zero_()
        graph.launch()
        torch.cuda.synchronize()
        # per-problem error against the float64 product of the bf16 values,
        # on every 16th problem
        errs_b = []
        for Ab, Bb, Cb in trip[::16]:
            refb = Ab.double() @ Bb.double()
            errs_b.append(float((Cb.double() - refb).norm() / refb.norm()))
        msb = timed_steps(graph.launch, max(3, args.steps // 2), 2, torch)
        graph.close()
        # the same products written as C = A B (MM_FLAG_OVERWRITE_C: C is
        # not read, plain stores), the form whose bytes count C once
        over = [sm.make_schedule(flags=sm.FLAG_OVERWRITE_C)] * len(trip)
        wso = torch.empty(sm.batched_workspace_bytes(trip, over), dtype=torch.uint8, device=dev)
        graph_o = sm.BatchedGraph(trip, schedules=over, workspace=wso)
        mso = timed_steps(graph_o.launch, max(3, args.steps // 2), 2, torch)
        graph_o.close()
        del wso
        att_o = sum(max(2.0 * m * n * k / (PEAK_BF16_TFLOPS * 1e12),
                        (2.0 * (m * k + k * n) + 4.0 * m * n) / (PEAK_HBM_GBS * 1e9)) for m, n, k in shapes)
        fl = sum(2.0 * m * n * k for m, n, k in shapes)
        batched_overwrite = {"ms": mso, "tflops": fl / (mso * 1e-3) / 1e12, "attainable_ms": att_o * 1e3,
                             "frac_of_attainable": att_o * 1e3 / mso}
        # attainable: each problem at its own roofline, the slower of bf16
        # MFMA peak and HBM for its unique bytes (A, B bf16 read once; fp32 C
        # read and written)
        att = sum(max(2.0 * m * n * k / (PEAK_BF16_TFLOPS * 1e12),
                      (2.0 * (m * k + k * n) + 8.0 * m * n) / (PEAK_HBM_GBS * 1e9)) for m, n, k in shapes)
        batched = {"problems": len(shapes), "ms": msb, "tflops": fl / (msb * 1e-3) / 1e12,
                   "flop": fl, "attainable_ms": att * 1e3, "frac_of_attainable": att * 1e3 / msb,
                   "max_rel_fro_err_sampled": max(errs_b), "error_target": 1e-5, "problems_checked": len(errs_b),
                   "overwrite_c": batched_overwrite,
                   "inputs": "bf16 N(0,1), m,n,k log-uniform [64,4096], fp32 accumulate"}
        # per-problem schedules chosen by the batch-aware autotuner (timing
        # the whole graph), against the library's own rule; and one Strassen
        # level on the largest problems, in the form that keeps the bf16
        # product's accuracy
        try:
            from paper_1911_05328_amd.tune import batch_tuner
            tuned_scheds, rep = batch_tuner.tune(trip, log=log)
            wst = torch.empty(max(sm.batched_workspace_bytes(trip, tuned_scheds), 1), dtype=torch.uint8, device=dev)
            graph_t = sm.BatchedGraph(trip, schedules=tuned_scheds, workspace=wst)
            mst = timed_steps(graph_t.launch, max(3, args.steps // 2), 2, torch)
            graph_t.close()
            del wst
            rep.pop("trace", None)
            batched["autotuned"] = {"ms": mst, "tflops": fl / (mst * 1e-3) / 1e12,
                                    "frac_of_attainable": att * 1e3 / mst, "tuner": rep}
            batched["strassen_check"] = batch_tuner.strassen_check(trip)
        except Exception as e:
            batched["autotuned"] = {"error": repr(e)}
        del trip, wsb
    except Exception as e:
        batched["error"] = repr(e)

    # the learned schedule proposal's regret, from the committed tuner report
    # (measured by tune/train.py on this GPU type, not in this run)
    learned = None
    try:
        rep = json.load(open(os.path.join(ROOT, "paper_1911_05328_amd", "tune", "costmodel_report_mi355x.json")))
        learned = {"source": "paper_1911_05328_amd/tune/costmodel_report_mi355x.json", "samples": rep["samples"],
                   "regret_mean": {k: rep[k]["mean"] for k in ("mlp", "mlp_top3", "default_no_mlp",
                                                              "planner_heuristic", "roofline_heuristic")
                                   if k in rep}}
    except Exception as e:
        learned = {"error": repr(e)}

    try:
        peaks = {k: v / 1e12 for k, v in sm.measured_peaks().items()}
    except Exception as e:
        peaks = {"error": repr(e)}
    roofline["frac_of_measured_peak"] = (achieved / peaks["mfma_bf16_flops"]) if achieved and \
        "mfma_bf16_flops" in peaks else None

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        cpu = cpu_baseline(depth, variant)
        cpu["reference_products_s"] = dict(oref.seconds) if oref is not None else None

    out = {
        "metric": METRIC, "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16" if prec == sm.PREC_FP16X3 else "bf16", "data": "synthetic",
        "step_events": step_stats,
        "config": {"workload": f"strassen_fp32target_n{N}", "m": N, "n": N, "k": N,
                   "strassen_depth": depth, "variant": "winograd" if variant else "classic",
                   "precision": PREC_DESC[prec], "inputs": "A, B iid N(0,1) fp32, seeds 1911/1912",
                   "rel_fro_err": err, "error_reference": err_kind, "error_detail": err_detail,
                   "error_target": TARGET_ERR,
                   "candidates": [{"depth": d, "variant": "winograd" if v else "classic",
                                   "precision": PREC_NAME[p], "rel_fro_err": e, "ms": t}
                                  for d, v, p, e, t in results]},
        "comparison": {"plain_dc_f32_n8192": {"ms": ms_plain, "tflops": tf_plain, "rel_fro_err": err_plain,
                                              "frac_f32_mfma_peak": tf_plain / PEAK_F32_TFLOPS},
                       "plain_dc_f32_n256_tile32": {"ms": ms_small, "tflops": 2.0 * 256 ** 3 / (ms_small * 1e-3) / 1e12,
                                                    "rel_fro_err": err_small, "error_target": 1e-6,
                                                    "oracle_ms": (cpu or {}).get("plain_dc_n256_ms"),
                                                    "note": "latency-bound: one launch of 64 workgroups"},
                       "speedup_vs_plain_dc": value / tf_plain,
                       "star_strassen_n8192": star,
                       "split_product_depth0_n8192": depth0_results,
                       "strassen_layouts_n8192": layouts,
                       "bilinear_n8192": bilinear,
                       "graph_replayed_step": graph_step,
                       "input_sets_and_fp64_additions": sets,
                       "learned_schedule_regret": learned,
                       "minplus_i32_n4096": secondary,
                       "batched_512_bf16_graph": batched},
        "roofline": roofline,
        "measured_peaks_T_per_s": peaks,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
