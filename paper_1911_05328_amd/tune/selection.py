"""Hand the tuner's results to the library so that calls without a schedule
use them (mm_cost_model_load, mm_tuned_load): the trained cost model's weights
and the measured timings of the DB, in the layouts the C ABI takes.  Host
marshalling only; the library evaluates the model and looks up the timings."""
from __future__ import annotations

import os

import numpy as np

import paper_1911_05328_amd as sm

from . import dataset, space

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "costmodel_mi355x.npz")


def accuracy_mask(path=MODEL_PATH):
    """The model's (3 x NSCHED) 0/1 accuracy mask (all ones if it has none)."""
    z = np.load(path)  # plain arrays only (no pickles)
    if "accurate" in z.files:
        return np.asarray(z["accurate"], np.float32).reshape(len(space.DTYPES), space.NSCHED)
    return np.ones((len(space.DTYPES), space.NSCHED), np.float32)


def model_params(path=MODEL_PATH):
    """Flat float32 parameters: t_mean, t_std, then W (out x in) and b per
    layer, then the accuracy mask (dtype-major)."""
    z = np.load(path)  # plain arrays only (no pickles)
    sizes = tuple(int(x) for x in z["sizes"])
    if sizes != (space.NFEAT, 64, 64, 64, space.NSCHED):
        raise ValueError(f"cost model of sizes {sizes} does not match the schedule space")
    parts = [np.array([float(z["t_mean"]), float(z["t_std"])], np.float32)]
    for l in range(len(sizes) - 1):
        parts += [np.asarray(z[f"W{l}"], np.float32).reshape(-1), np.asarray(z[f"b{l}"], np.float32).reshape(-1)]
    parts.append(accuracy_mask(path).reshape(-1))
    return np.concatenate(parts)


def timing_entries(rows):
    """(semiring, dtype, m, n, k, Schedule, ms) for every measured schedule of
    the DB rows within the error target, the in-kernel-split variants
    included."""
    out = []
    for r in rows:
        sr, dt = space.semiring_and_dtype(r["dtype"])
        m, n, k = r["m"], r["n"], r["k"]
        ik = r.get("times_inkernel_ms") or [None] * space.NSCHED
        for j in range(space.NSCHED):
            if not dataset.within_target(r, j):
                continue
            if r["times_ms"][j] is not None:
                out.append((sr, dt, m, n, k, space.schedule(r["dtype"], m, j), float(r["times_ms"][j])))
            if ik[j] is not None:
                out.append((sr, dt, m, n, k, space.schedule(r["dtype"], m, j, inkernel=True), float(ik[j])))
    return out


def load(model_path=MODEL_PATH, db_path=dataset.DB_PATH) -> None:
    """Load the cost model and/or the timings (either path may be None)."""
    if model_path:
        sm.cost_model_load(model_params(model_path))
    if db_path:
        sm.tuned_load(timing_entries(dataset.load_db(db_path)))
