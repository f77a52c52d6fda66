"""Train the cost model on the timing DB (GPU, the library's kernels) and
report its regret on the held-out shapes against exhaustive search within
the error target, the default schedule and the planner's and roofline
heuristics.

Run: python -m paper_1911_05328_amd.tune.train [--db PATH] [--out WEIGHTS.npz] [--report REPORT.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import dataset, propose, space
from .mlp import CostModel


def evaluate(model, rows, X, F, TT, meta, TTacc, topk=3):
    """Regrets on held-out samples.  F / TT: workspace feasibility and times
    of every schedule; TTacc: the same times with schedules measured above
    the error target on that very row set to inf.  The picks see only the
    workspace feasibility and the model's accuracy mask (learned from the
    training rows); regret is against the fastest schedule that fits and
    meets the target (exhaustive search over TTacc), and `violations`
    counts picks whose measured error on the held-out row is above it."""
    mask = getattr(model, "accurate", None)
    allowed = F > 0
    if mask is not None:
        allowed = allowed & np.array([mask[space.DTYPES.index(rows[ri]["dtype"])] > 0 for ri, _ in meta])
    pred = np.where(allowed, model.predict(X), np.inf)
    order = np.argsort(pred, axis=1)
    pick = order[:, 0]
    # top-k refinement: the best measured time among the model's k best
    topk_pick = np.array([min(order[i, :topk], key=lambda j: TT[i, j]) for i in range(len(pick))])
    default = np.full(len(pick), dataset.DEFAULT_IDX)
    heur = np.array([propose.heuristic(rows[ri]["m"], rows[ri]["n"], rows[ri]["k"], rows[ri]["dtype"], b, allowed[i])
                     for i, (ri, b) in enumerate(meta)])
    roof = np.array([propose.roofline_heuristic(rows[ri]["m"], rows[ri]["n"], rows[ri]["k"], rows[ri]["dtype"],
                                                allowed[i])
                     for i, (ri, b) in enumerate(meta)])

    def reg(p):
        t = TT[np.arange(len(p)), p]
        return t / TTacc.min(axis=1) - 1.0

    def viol(p):
        return int(np.sum(~np.isfinite(TTacc[np.arange(len(p)), p]) & np.isfinite(TT[np.arange(len(p)), p])))

    out = {"mlp": dataset.summary(reg(pick)),
           f"mlp_top{topk}": dataset.summary(reg(topk_pick)),
           "default_no_mlp": dataset.summary(reg(default)),
           "planner_heuristic": dataset.summary(reg(heur)),
           "roofline_heuristic": dataset.summary(reg(roof)),
           "exhaustive": dataset.summary(reg(TTacc.argmin(axis=1))),
           "violations": {"mlp": viol(pick), f"mlp_top{topk}": viol(topk_pick), "default_no_mlp": viol(default),
                          "roofline_heuristic": viol(roof)},
           "error_target": space.TARGET_ERROR,
           "samples": int(len(pick))}
    return out


def run(db=dataset.DB_PATH, steps=2000, seed=1911, out=None, report=None, log=print):
    rows = dataset.load_db(db)
    train = [r for r in rows if r["split"] == "train"]
    test = [r for r in rows if r["split"] == "test"]
    Xtr, Ttr, Ftr, _, _ = dataset.samples(train, 4, seed)
    Xte, _, Fte, TTte, meta = dataset.samples(test, 4, seed + 1, max_error=None)
    _, _, _, TTacc, _ = dataset.samples(test, 4, seed + 1)
    model = CostModel(seed=seed)
    model.accurate = dataset.accuracy_mask(train)
    t0 = time.time()
    hist = model.fit(Xtr, Ttr, Ftr, steps=steps, log_every=max(steps // 10, 1))
    train_s = time.time() - t0
    rep = evaluate(model, test, Xte, Fte, TTte, meta, TTacc)
    rep["train"] = {"samples": int(len(Xtr)), "steps": steps, "seconds": train_s, "loss_history": hist}
    rep["db"] = {"rows": len(rows), "train_rows": len(train), "test_rows": len(test)}
    rep["accuracy_mask"] = {d: [int(v) for v in model.accurate[i]] for i, d in enumerate(space.DTYPES)}
    if out:
        model.save(out)
    if report:
        json.dump(rep, open(report, "w"), indent=1)
    log(json.dumps({k: v for k, v in rep.items() if k != "train"}, indent=1))
    log(f"training: {len(Xtr)} samples, {steps} steps, {train_s:.1f} s, loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
    return model, rep


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--db", default=dataset.DB_PATH)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=1911)
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    run(a.db, a.steps, a.seed, a.out, a.report)
    return 0


if __name__ == "__main__":
    sys.exit(main())
