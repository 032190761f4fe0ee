"""Learned step-time cost model: harvesting, training and tile choice.

The paper ranks contraction candidates by their measured time on the device
(Sec. 4.1) and scores contraction trees with a cost that weighs compute and
memory traffic (Sec. 3.2).  Here the cost of one kernel launch of a step is
learned: the library's HIP kernels train a 2 x 64 ReLU MLP (tn_costmodel_*) on
ln(microseconds) of steps timed with HIP events on the plan's stream
(tn_plan_step_times), from the step features the library computes
(tn_plan_step_features, layout in include/tn.h).  A trained model picks every
MFMA step's tile shape (tn_plan_tune_with_model) without timing the candidates,
and sums to a predicted plan time for comparing plans built on the host only
(for instance different slicings of one network).

This module only marshals arrays: features, training, prediction and tile
choice all run in the library.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import tn

N_FEATURES = tn.TN_COST_FEATURES
FEATURE_NAMES = [
    "batch_bits", "m_bits", "n_bits", "k_bits", "log2_flops", "log2_bytes", "log2_intensity",
    "grid_m_bits", "grid_n_bits", "log2_splits", "log2_blocks", "per_slice",
    "k_small", "k_mfma_f32", "k_mfma_f16x3", "k_mfma_bf16x3",
    "tile_256x128", "tile_128x128", "tile_128x64", "tile_64x64",
    "a_contig", "b_contig", "c_contig", "a_split", "b_split", "c_split",
    "m_tile_shortfall", "n_tile_shortfall", "log2_k_stages",
]
assert len(FEATURE_NAMES) == N_FEATURES

DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                             "costmodel_mi355x.json")


class CostModel:
    """Owning wrapper of a tn_costmodel handle (parameters live on the GPU)."""

    handle = None

    def __init__(self, n_features: int = N_FEATURES, seed: int = 0):
        self.handle = tn.tn_costmodel_create(n_features, seed)
        self.n_features, self.hidden, self.n_params = tn.tn_costmodel_describe(self.handle)
        self.mean = np.zeros(n_features, np.float32)
        self.std = np.ones(n_features, np.float32)

    def close(self):
        if getattr(self, "handle", None):
            tn.tn_costmodel_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- parameters ---------------------------------------------------------
    def params(self) -> np.ndarray:
        return tn.tn_costmodel_get_params(self.handle, self.n_params)

    def set_params(self, theta):
        tn.tn_costmodel_set_params(self.handle, theta)

    def set_normalization(self, mean, std):
        self.mean = np.asarray(mean, np.float32).copy()
        self.std = np.asarray(std, np.float32).copy()
        tn.tn_costmodel_set_normalization(self.handle, self.mean, self.std)

    # -- evaluation and training -------------------------------------------
    def predict(self, X) -> np.ndarray:
        """Raw outputs (ln microseconds for the step-time model)."""
        return tn.tn_costmodel_predict(self.handle, X)

    def predict_us(self, X) -> np.ndarray:
        return np.exp(self.predict(X).astype(np.float64))

    def gradient(self, X, t):
        """(gradient, loss) of the mean squared error over the rows of X."""
        return tn.tn_costmodel_gradient(self.handle, X, t)

    def adam_step(self, grad, lr: float):
        tn.tn_costmodel_adam_step(self.handle, grad, lr)

    def train(self, X, t, epochs: int, batch: int, lr: float, seed: int = 0) -> float:
        return tn.tn_costmodel_train(self.handle, X, t, epochs, batch, lr, seed)

    def fit(self, X, us, epochs: int = 400, batch: int = 256, lr: float = 2e-3,
            seed: int = 0) -> float:
        """Standardise the features of X and train on ln(us); returns the final MSE."""
        X = np.asarray(X, np.float32)
        mean = X.mean(axis=0)
        std = X.std(axis=0)
        std = np.where(std > 1e-6, std, 1.0).astype(np.float32)
        self.set_normalization(mean, std)
        return self.train(X, np.log(np.asarray(us, np.float64)).astype(np.float32),
                          epochs, batch, lr, seed)

    # -- persistence ----------------------------------------------------------
    def save(self, path: str, meta: dict | None = None):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        doc = {"n_features": self.n_features, "hidden": self.hidden,
               "feature_names": FEATURE_NAMES[:self.n_features],
               "mean": self.mean.tolist(), "std": self.std.tolist(),
               "params": self.params().tolist(), "meta": meta or {}}
        with open(path, "w") as f:
            json.dump(doc, f)

    @classmethod
    def load(cls, path: str = DEFAULT_MODEL) -> "CostModel":
        with open(path) as f:
            doc = json.load(f)
        m = cls(int(doc["n_features"]))
        m.set_normalization(doc["mean"], doc["std"])
        m.set_params(np.asarray(doc["params"], np.float32))
        m.meta = doc.get("meta", {})
        return m


def predict_plan_us(plan, model: CostModel, n_slices: int | None = None) -> float:
    """Predicted microseconds of contracting n_slices slices (default: all) with the plan's
    tiles chosen by the model: slice-independent steps once, slice-dependent steps once per
    chunk of slice_batch slices.  Works on host-only plans."""
    pred = plan.tune_with_model(model)
    info = plan.describe()
    n = info["n_slices"] if n_slices is None else n_slices
    chunks = -(-n // max(info["slice_batch"], 1))
    total = 0.0
    for us, st in zip(pred, plan.steps()):
        total += float(us) * (chunks if st["per_slice"] else 1)
    return total


class StepTimeTable:
    """The model's time of a pairwise step by its (m, n, k) bit counts, for scoring contraction
    trees by predicted time (planner.refine(step_time=...)).  A step is the library's canonical
    step of those extents (tn_costmodel_predict_shapes: k innermost in both operands, the
    planner's kernel, the fastest predicted tile) with `batch_bits` batch bits; both operand
    orders are asked and the faster kept.  Answers are cached; prefill() asks many shapes in
    one forward pass."""

    def __init__(self, model: CostModel, precision="f16x3", batch_bits: int = 0, floor_rate: float | None = None):
        """floor_rate (flop/s), when given, bounds every step's time from below by its flops
        (8 real flops per complex multiply-add) at that rate, so that an annealer scored by
        the table cannot favour steps the model predicts faster than, for instance, its own
        prediction for a large balanced step (large_step_rate())."""
        self.model, self.precision, self.batch_bits = model, precision, int(batch_bits)
        self.floor_rate = floor_rate
        self.cache = {}

    def prefill(self, shapes):
        todo = sorted({(int(m), int(n), int(k)) for m, n, k in shapes} - set(self.cache))
        if not todo:
            return
        rows = []
        for m, n, k in todo:
            rows.append((self.batch_bits, m, n, k))
            rows.append((self.batch_bits, n, m, k))
        us = tn.tn_costmodel_predict_shapes(self.model.handle, self.precision, rows)
        for i, (m, n, k) in enumerate(todo):
            t = float(min(us[2 * i], us[2 * i + 1]))
            if self.floor_rate:
                t = max(t, 8.0 * 2.0 ** (self.batch_bits + m + n + k) / self.floor_rate * 1e6)
            self.cache[(m, n, k)] = t

    def large_step_rate(self, bits: int = 13) -> float:
        """flop/s the model predicts for a large balanced step (2^bits x 2^bits x 2^(bits-1))."""
        us = self(bits, bits, bits - 1)
        return 8.0 * 2.0 ** (self.batch_bits + 3 * bits - 1) / (us * 1e-6)

    def __call__(self, m: int, n: int, k: int) -> float:
        key = (int(m), int(n), int(k))
        if key not in self.cache:
            self.prefill([key])
        return self.cache[key]


# MI355X roofline of the analytic model: dense MFMA peaks (FP32 for the complex64 GEMM,
# FP16 / BF16 for the split form, whose three products each run the step's flops), FP32
# vector for the small kernel, HBM3E bandwidth.
PEAK_FP32 = 157.3e12
PEAK_SPLIT = 2.5e15 / 3
HBM_BW = 8.0e12


def analytic_step_us(step: dict) -> float:
    """Roofline time of one step for one slice (or once, if slice-independent):
    max(flops / peak, bytes / bandwidth), with the peak of the step's kernel."""
    rate = PEAK_SPLIT if step["kernel"] in (2, 3) else PEAK_FP32
    return max(step["flops"] / rate, step["bytes"] / HBM_BW) * 1e6


def analytic_plan_us(plan, n_slices: int | None = None) -> float:
    """Analytic flop/byte estimate of contracting n_slices slices (default: all): the
    fallback the learned model is compared with.  Works on host-only plans."""
    info = plan.describe()
    n = info["n_slices"] if n_slices is None else n_slices
    return sum(analytic_step_us(st) * (n if st["per_slice"] else 1) for st in plan.steps())


# ---------------------------------------------------------------------------
# Harvesting
# ---------------------------------------------------------------------------
def step_tile_ids(plan) -> list:
    """Current tile id of every step (-1 for steps on the small kernel)."""
    return [s["tile"] for s in plan.steps()]


def harvest(plan, tiles=(0, 1, 2, 3), n_slices: int | None = None, reps: int = 3,
            tag: str = "") -> list:
    """Time every step of a device plan (created with record_steps=True) with each
    tile id, over slices [0, n_slices) (default: one chunk).

    Returns records {"tag", "step", "tile", "kernel", "features", "us"} with the
    mean microseconds per launch.  Restores the plan's tiles and clears its
    accumulator afterwards.
    """
    info = plan.describe()
    if n_slices is None:
        n_slices = min(info["n_slices"], info["slice_batch"])
    steps = plan.steps()
    before = step_tile_ids(plan)
    mfma = [i for i, s in enumerate(steps) if s["kernel"] != 0]
    out = []
    for ti, t in enumerate(tiles):
        for i in mfma:
            plan.set_tile(i, t)
        plan.contract(0, n_slices)         # warm-up
        plan.step_times()
        for _ in range(reps):
            plan.contract(0, n_slices)
        ms, cnt = plan.step_times()
        for i, s in enumerate(steps):
            if cnt[i] == 0 or (s["kernel"] == 0 and ti > 0):
                continue
            tile = t if s["kernel"] != 0 else -1
            out.append({"tag": tag, "step": i, "tile": tile, "kernel": s["kernel"],
                        "features": plan.step_features(i, tile).tolist(),
                        "us": 1e3 * float(ms[i]) / int(cnt[i])})
    for i in mfma:
        plan.set_tile(i, before[i])
    plan.reset()
    return out


def records_to_arrays(records):
    X = np.asarray([r["features"] for r in records], np.float32)
    us = np.asarray([r["us"] for r in records], np.float64)
    return X, us


def tile_choice_report(records, model: CostModel, default_tiles: dict) -> dict:
    """Compare, per (tag, step) measured with every tile, the measured time of the
    model's argmin tile with the default (heuristic) tile and the fastest tile; also
    summed over only the steps where the model's and the heuristic's tiles differ.

    default_tiles maps (tag, step) -> tile id the shape heuristic picks.
    """
    groups = {}
    for r in records:
        if r["tile"] < 0:
            continue
        groups.setdefault((r["tag"], r["step"]), []).append(r)
    tot = {"model": 0.0, "heuristic": 0.0, "best": 0.0, "worst": 0.0,
           "model_where_differ": 0.0, "heuristic_where_differ": 0.0}
    n = 0
    hits = 0
    differ = 0
    for key, rs in groups.items():
        if len(rs) < 2 or key not in default_tiles:
            continue
        X = np.asarray([r["features"] for r in rs], np.float32)
        pred = model.predict(X)
        meas = np.asarray([r["us"] for r in rs])
        tiles = [r["tile"] for r in rs]
        if default_tiles[key] not in tiles:
            continue
        pick = int(np.argmin(pred))
        heur = tiles.index(default_tiles[key])
        tot["model"] += meas[pick]
        tot["heuristic"] += meas[heur]
        if pick != heur:
            differ += 1
            tot["model_where_differ"] += meas[pick]
            tot["heuristic_where_differ"] += meas[heur]
        tot["best"] += meas.min()
        tot["worst"] += meas.max()
        hits += int(meas[pick] <= meas.min() * 1.05)
        n += 1
    tot["steps"] = n
    tot["differ"] = differ
    tot["within_5pct_of_best"] = hits
    return tot
