"""Learned planner cost model (GPU-trained perceptron) and its evaluation.

The perceptron (qw_mlp_* kernels of libqw: BF16 matrix-core products, FP32
accumulation, FP32 master weights and Adam) maps the 12 planner features of
a workload (`cost_study.features`) to two standardized targets learned from
the realized costs the simulator logs (`cost_study`):
    y0 = log(t_direct / t_reuse) - log(r_analytic),   y1 = log t_reuse [ms],
where r_analytic is the byte-count ratio of Eq. (2)'s analytic estimates
(feature 10). The network thus learns the correction to the analytic model
where realized times depart from byte counts (launch latency at small n,
caching of the shared snapshot). Its decision is guarded like Eq. (2):
reuse iff r_analytic * exp(y0) > 1 + delta_L, with delta_L chosen on the
training split (the analytic rule keeps the paper's delta = 0.10). It
abstains without asking the network when the workload has no shared
prefix, and falls back to the analytic rule when a feature lies outside the
range seen in training. Results never depend on it: a plan only changes
timing.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import binding as B

N_IN, N_OUT, N_PARAMS = 12, 2, 5122
DELTA = 0.10
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "c5_costs.jsonl")


def load_costs(path: str = DATA) -> List[dict]:
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def split(rows: Sequence[dict], n_test: int = 400, seed: int = 505) -> Tuple[list, list]:
    """Seeded held-out split (1600 / 400 for the 2000-workload study)."""
    perm = np.random.default_rng(seed).permutation(len(rows))
    test = set(int(i) for i in perm[:n_test])
    return [r for i, r in enumerate(rows) if i not in test], [r for i, r in enumerate(rows) if i in test]


def analytic_log_ratio(features: Sequence[float]) -> float:
    """log of the analytic estimate est_direct / est_reuse (feature 10 holds
    the ratio / 10, capped at 20)."""
    return math.log(max(features[10] * 10.0, 1e-3))


def arrays(rows: Sequence[dict]) -> Tuple[np.ndarray, np.ndarray]:
    """Features and raw targets (log-ratio correction, log t_reuse)."""
    x = np.array([r["features"] for r in rows], dtype=np.float32)
    y = np.array([[math.log(r["t_direct_ms"] / r["t_reuse_ms"]) - analytic_log_ratio(r["features"]),
                   math.log(r["t_reuse_ms"])] for r in rows], dtype=np.float32)
    return x, y


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (the layout of qw.h)."""
    g = np.random.default_rng(seed)
    parts = []
    for k, n in ((N_IN, 64), (64, 64), (64, N_OUT)):
        lim = math.sqrt(6.0 / k)
        parts += [g.uniform(-lim, lim, size=k * n), np.zeros(n)]
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """Device-resident perceptron: parameters, Adam moments, workspace."""

    def __init__(self, ctx, params: Optional[np.ndarray] = None, seed: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        dev = f"cuda:{ctx.device}"
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        self.p = torch.tensor(p, device=dev)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.step = 0
        self._work = None
        self.x_lo = self.x_hi = None   # training feature range (fallback test)
        self.y_mu = np.zeros(N_OUT, dtype=np.float32)   # target standardization
        self.y_sd = np.ones(N_OUT, dtype=np.float32)
        self.delta = DELTA             # decision guard, calibrated by train()

    def _ws(self, batch: int):
        need = int(B.lib().qw_mlp_workspace_floats(batch))
        if self._work is None or self._work.numel() < need:
            self._work = self.torch.empty(need, dtype=self.torch.float32, device=self.p.device)
        return self._work

    def forward(self, x_dev, y_dev=None):
        bsz = int(x_dev.shape[0])
        if y_dev is None:
            y_dev = self.torch.empty((bsz, N_OUT), dtype=self.torch.float32, device=self.p.device)
        self.ctx.check(B.lib().qw_mlp_forward(self.ctx.h, self.p.data_ptr(), x_dev.data_ptr(), bsz,
                                              self._ws(bsz).data_ptr(), y_dev.data_ptr()))
        return y_dev

    def backward(self, x_dev, t_dev):
        bsz = int(x_dev.shape[0])
        self.ctx.check(B.lib().qw_mlp_backward(self.ctx.h, self.p.data_ptr(), x_dev.data_ptr(),
                                               t_dev.data_ptr(), bsz, self._ws(bsz).data_ptr(),
                                               self.g.data_ptr()))
        return self.g

    def backward_rows(self, x_dev, t_dev, rows: np.ndarray):
        """Gradient on the mini-batch of rows `rows` (host indices) of the
        device arrays x_dev, t_dev: the library gathers them in its kernels."""
        import ctypes
        rows = np.ascontiguousarray(rows, dtype=np.uint32)
        bsz = len(rows)
        self.ctx.check(B.lib().qw_mlp_backward_rows(
            self.ctx.h, self.p.data_ptr(), x_dev.data_ptr(), t_dev.data_ptr(), int(x_dev.shape[0]),
            ctypes.c_void_p(rows.ctypes.data), bsz, self._ws(bsz).data_ptr(), self.g.data_ptr()))
        return self.g

    def adam(self, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        self.ctx.check(B.lib().qw_mlp_adam(self.ctx.h, self.p.data_ptr(), self.g.data_ptr(),
                                           self.m.data_ptr(), self.v.data_ptr(), self.step, lr, b1,
                                           b2, eps))

    def train(self, x: np.ndarray, y: np.ndarray, epochs: int = 300, batch: int = 256,
              lr: float = 3e-3, seed: int = 1) -> Dict[str, float]:
        """Mini-batch Adam on the GPU kernels (standardized targets); returns
        timing and losses."""
        torch = self.torch
        dev = self.p.device
        self.y_mu, self.y_sd = y.mean(axis=0), np.maximum(y.std(axis=0), 1e-6)
        xd = torch.tensor(x, device=dev)
        yd = torch.tensor((y - self.y_mu) / self.y_sd, device=dev)
        self.x_lo, self.x_hi = x.min(axis=0), x.max(axis=0)
        n = len(x)
        g = np.random.default_rng(seed)
        first = self.loss(xd, yd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(epochs):
            perm = g.permutation(n)
            for s in range(0, n, batch):
                self.backward_rows(xd, yd, perm[s:s + batch])
                self.adam(lr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return {"epochs": epochs, "s_per_epoch": dt / max(1, epochs), "loss_initial": first,
                "loss_final": self.loss(xd, yd)}

    def loss(self, xd, yd) -> float:
        """1/(2B) sum (y - t)^2 over all rows (the library's loss kernel)."""
        bsz = int(xd.shape[0])
        out = self.torch.empty(1, dtype=self.torch.float64, device=self.p.device)
        self.ctx.check(B.lib().qw_mlp_loss(self.ctx.h, self.p.data_ptr(), xd.data_ptr(), yd.data_ptr(),
                                           bsz, self._ws(bsz).data_ptr(), out.data_ptr()))
        return float(out.cpu().item())

    def predict(self, x: np.ndarray) -> np.ndarray:
        """Raw targets (log-ratio correction, log t_reuse) for features x."""
        xd = self.torch.tensor(np.asarray(x, dtype=np.float32), device=self.p.device)
        return self.forward(xd).cpu().numpy() * self.y_sd + self.y_mu

    def calibrate(self, rows: Sequence[dict], grid=(0.0, 0.01, 0.02, 0.05, 0.1)) -> float:
        """Pick the decision guard with the least realized regret on `rows`
        (the training split); ties go to the larger guard."""
        pred = self.predict(arrays(rows)[0])
        best = None
        for d in grid:
            self.delta = d
            reg = float(np.mean([_regret(r, mlp_reuse(self, r["features"], r["negative"], p)[0])
                                 for r, p in zip(rows, pred)]))
            if best is None or reg <= best[0]:
                best = (reg, d)
        self.delta = best[1]
        return self.delta

    def in_range(self, f: np.ndarray) -> bool:
        if self.x_lo is None:
            return False
        return bool(np.all(f >= self.x_lo - 1e-6) and np.all(f <= self.x_hi + 1e-6))


# ---------------------------------------------------------------- decisions
def analytic_reuse(features: Sequence[float], negative: bool, delta: float = DELTA) -> bool:
    """Eq. (2) on the analytic byte estimates carried by the features:
    reuse iff est_direct > (1 + delta) est_reuse."""
    if negative:
        return False
    ratio = features[10] * 10.0
    return ratio > 1.0 + delta


def mlp_reuse(model: MLP, features: Sequence[float], negative: bool,
              pred: Optional[np.ndarray] = None) -> Tuple[bool, str]:
    if negative:
        return False, "no shared prefix"
    f = np.asarray(features, dtype=np.float32)
    if not model.in_range(f):
        return analytic_reuse(features, negative), "fallback: features outside the training range"
    p = pred if pred is not None else model.predict(f[None, :])[0]
    log_ratio = analytic_log_ratio(features) + float(p[0])
    return bool(log_ratio > math.log1p(model.delta)), "learned model"


def _regret(r: dict, reuse: bool) -> float:
    td, tr = r["t_direct_ms"], r["t_reuse_ms"]
    best = min(td, tr)
    return ((tr if reuse else td) - best) / best


def planner_hook(model: MLP):
    """A `decide` callback for planner.plan_workload: the learned decision
    at a trie node (None, i.e. the analytic rule, out of range)."""
    from .cost_study import feature_vector

    def decide(node, info):
        sb2 = 2.0 * info["state_bytes"]
        f = feature_vector(info["n"], info["tasks"], info["c_prefix"] / sb2,
                           [c / sb2 for c in info["suffix_costs"]], info["prefix_gates"],
                           info["suffix_gates"])
        reuse, why = mlp_reuse(model, f, negative=info["c_prefix"] <= 0.0)
        return None if why.startswith("fallback") else reuse
    return decide


def evaluate(model: MLP, rows: Sequence[dict]) -> Dict[str, float]:
    """Plan regret and abstention accuracy of the learned and analytic
    decisions on realized costs (truth: abstain iff direct <= reuse)."""
    x, _ = arrays(rows)
    pred = model.predict(x)
    out = {}
    for name in ("mlp", "analytic", "analytic_delta0"):
        regret, correct, neg_ok, neg_n, fallbacks = [], 0, 0, 0, 0
        for r, pr in zip(rows, pred):
            if name == "mlp":
                reuse, why = mlp_reuse(model, r["features"], r["negative"], pr)
                fallbacks += why.startswith("fallback")
            else:
                reuse = analytic_reuse(r["features"], r["negative"],
                                       DELTA if name == "analytic" else 0.0)
            td, tr = r["t_direct_ms"], r["t_reuse_ms"]
            regret.append(_regret(r, reuse))
            truth_abstain = td <= tr
            correct += (not reuse) == truth_abstain
            if r["negative"]:
                neg_n += 1
                neg_ok += not reuse
        out[name] = {"regret_mean": float(np.mean(regret)), "regret_max": float(np.max(regret)),
                     "abstain_accuracy": correct / len(rows),
                     "negative_control_abstain": neg_ok / max(1, neg_n), "fallbacks": fallbacks}
    return out


def train_and_evaluate(ctx, path: str = DATA, epochs: int = 300, seed: int = 0) -> dict:
    rows = load_costs(path)
    train_rows, test_rows = split(rows)
    x, y = arrays(train_rows)
    model = MLP(ctx, seed=seed)
    stats = model.train(x, y, epochs=epochs)
    stats["delta"] = model.calibrate(train_rows)
    xt, yt = arrays(test_rows)
    # inference latency for one decision
    f1 = xt[:1]
    model.predict(f1)
    t0 = time.perf_counter()
    for _ in range(20):
        model.predict(f1)
    infer_us = (time.perf_counter() - t0) / 20 * 1e6
    res = evaluate(model, test_rows)
    res["train"] = stats
    res["inference_us"] = infer_us
    res["n_train"], res["n_test"] = len(train_rows), len(test_rows)
    res["test_rmse_log"] = [float(v) for v in np.sqrt(np.mean((model.predict(xt) - yt) ** 2, axis=0))]
    return {"model": model, "report": res}
