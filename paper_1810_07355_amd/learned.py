"""Learned per-query search range: labels from eps sweeps, training of the
2-layer perceptron with the library's kernels (column statistics and
z-scoring, forward/backward, Adam, the fold of the target scaling into the
output layer), and calibration of the per-target shift.  Not part of the
paper; the plain eps sweep stays the fallback and the measure of recall.

Model: 14 features of the state after the probe expansions -> 64 ReLU ->
heads.  Log-eps mode: one head per target (or per (k, target) class), each
predicting log10(eps + 0.01) of the smallest grid eps at which the query
reaches that recall.  Curve mode: for each candidate range, the query's
recall and log(1 + cost) there, the cost being its distance computations or
its search time (time_cost)."""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import _lib as L
from . import api

EPS_OFFSET = 0.01


def eps_to_target(eps):
    return np.log10(np.asarray(eps, dtype=np.float64) + EPS_OFFSET)


def dynamic_ep(eps: float, e0: float = 30.0, we: float = 20.0) -> int:
    """Equation 1, e_p = 10^(w_e eps) + e_0, as an edge count."""
    return int(min(math.floor(10.0 ** (we * float(np.float32(eps))) + e0), L.EP_INF))


def recall_by_ids(ids: np.ndarray, gt_ids: np.ndarray, k: int) -> np.ndarray:
    """Per-query recall@k: returned ids found among the k true neighbours."""
    ids = ids[:, :k]
    gt = gt_ids[:, :k]
    hit = (ids[:, :, None] == gt[:, None, :]).any(axis=2) & (ids >= 0)
    return hit.sum(axis=1) / float(k)


def labels_from_recalls(recalls: np.ndarray, grid, targets) -> np.ndarray:
    """recalls[e, q] at grid[e] -> per query and target the smallest grid eps
    reaching the target (the largest grid eps if none does)."""
    grid = np.asarray(grid, dtype=np.float64)
    out = np.empty((recalls.shape[1], len(targets)))
    for t, tgt in enumerate(targets):
        reach = recalls >= tgt - 1e-9
        idx = np.where(reach.any(axis=0), reach.argmax(axis=0), len(grid) - 1)
        out[:, t] = grid[idx]
    return out


@dataclasses.dataclass
class Trained:
    W1: torch.Tensor
    b1: torch.Tensor
    W2: torch.Tensor
    b2: torch.Tensor
    mean: torch.Tensor
    std: torch.Tensor
    losses: list

    def predictor(self, head=0, shift=None, eps_min=0.0, eps_max=0.5, e0=30.0, we=20.0,
                  head_per_query=None, mode=L.PRED_LOG_EPS, eps_cand=None, lam=0.0,
                  lambda_per_query=None) -> api.Predictor:
        dev = self.W1.device
        if shift is None and mode == L.PRED_LOG_EPS:
            shift = torch.zeros(self.W2.shape[0], dtype=torch.float32, device=dev)
        cand = None
        if eps_cand is not None:
            cand = torch.as_tensor(np.asarray(eps_cand, dtype=np.float32), device=dev)
        return api.Predictor(api.to_bf16_bits(self.W1), self.b1, api.to_bf16_bits(self.W2),
                             self.b2, self.mean, self.std, shift=shift, head=head,
                             head_per_query=head_per_query, eps_min=eps_min, eps_max=eps_max,
                             e0=e0, we=we, mode=mode, eps_cand=cand, lam=lam,
                             lambda_per_query=lambda_per_query)


def train_targets(features: torch.Tensor, Y: np.ndarray, metric: int, hidden: int = 64,
                  steps: int = 4000, batch: int = 1024, lr: float = 3e-3, seed: int = 0,
                  weights: np.ndarray | None = None) -> Trained:
    """Fit the perceptron to targets Y [n, T] (mean squared error, each target
    column standardised during training and folded back into the last layer).
    features: raw [n, 14] f32 on the GPU.  weights [n, T] (optional): the
    weight of each target in the loss, e.g. one-hot when each sample labels
    only its own head; the standardisation then uses the weighted moments."""
    dev = features.device
    X = api.feature_transform(features.contiguous(), metric)
    mean_t, std_t = api.column_stats(X)
    Xz = api.standardize(X, mean_t, std_t)
    Yd = torch.from_numpy(np.asarray(Y, dtype=np.float32)).to(dev)
    Wt = None if weights is None else torch.from_numpy(np.asarray(weights, dtype=np.float32)).to(dev)
    ym_t, ys_t = api.column_stats(Yd, Wt)
    Yt = api.standardize(Yd, ym_t, ys_t)
    n, F = Xz.shape
    T = Yt.shape[1]
    g = np.random.default_rng(seed)
    W1 = torch.from_numpy((g.standard_normal((hidden, F)) * math.sqrt(2.0 / F)).astype(np.float32)).to(dev)
    b1 = torch.zeros(hidden, dtype=torch.float32, device=dev)
    W2 = torch.from_numpy((g.standard_normal((T, hidden)) * math.sqrt(1.0 / hidden)).astype(np.float32)).to(dev)
    b2 = torch.zeros(T, dtype=torch.float32, device=dev)
    params = [W1, b1, W2, b2]
    ms = [torch.zeros_like(p) for p in params]
    vs = [torch.zeros_like(p) for p in params]
    losses = []
    batch = min(batch, n)
    perm = g.permutation(n)
    pos = 0
    for t in range(1, steps + 1):
        if pos + batch > n:
            perm = g.permutation(n)
            pos = 0
        idx = torch.from_numpy(perm[pos:pos + batch]).to(dev)
        pos += batch
        xb = Xz.index_select(0, idx).contiguous()
        yb = Yt.index_select(0, idx).contiguous()
        wb = None if Wt is None else Wt.index_select(0, idx).contiguous()
        loss, grads = api.mlp_backward(xb, yb, W1, b1, W2, b2, w=wb)
        step_lr = lr * (0.5 * (1.0 + math.cos(math.pi * t / steps)) * 0.9 + 0.1)
        for p, gr, m, v in zip(params, grads, ms, vs):
            api.adam_step(p, gr, m, v, step_lr, t)
        if t % 100 == 0 or t == 1:
            losses.append(float(loss.item()))
    # fold the target standardisation into the last layer
    api.mlp_fold_output(W2, b2, ys_t, ym_t)
    return Trained(W1, b1, W2, b2, mean_t, std_t, losses)


def train(features: torch.Tensor, labels: np.ndarray, metric: int, **kw) -> Trained:
    """Log-range heads: each target recall's smallest sufficient eps."""
    return train_targets(features, eps_to_target(labels), metric, **kw)


def curve_targets(recalls: np.ndarray, cost: np.ndarray, cand_idx) -> np.ndarray:
    """[n, 2G]: recall at each candidate range, then log(1 + cost) there
    (recalls, cost: [n_eps, n]; the cost is the distance computations, or
    time_cost of the queries' search times)."""
    cand_idx = list(cand_idx)
    return np.concatenate([recalls[cand_idx].T, np.log1p(cost[cand_idx].T.astype(np.float64))],
                          axis=1)


def time_cost(us: np.ndarray, dcs: np.ndarray) -> np.ndarray:
    """Per-query search time in units of distance computations: each
    query's device time at each range (the search's own per-query clock),
    scaled so that the sweep's total equals its total distance computations.
    A query's time follows its expansions about as much as its distance
    computations (each expansion costs a fixed sequence of marks, sorts and
    merges), so a range chosen by time favours queries whose expansions still
    yield new nodes; the scale keeps a budget relative to the cost in the
    units of max_dc."""
    us = np.asarray(us, dtype=np.float64)
    scale = float(np.asarray(dcs, dtype=np.float64).sum()) / max(float(us.sum()), 1e-30)
    return us * scale


def calibrate(run_recall, target: float, lo: float = -1.0, hi: float = 1.0, iters: int = 9,
              slack: float = 0.0) -> tuple[float, float]:
    """Smallest shift (log10 units) whose mean recall reaches target + slack;
    run_recall(shift) -> mean recall is monotone in the shift up to noise."""
    goal = target + slack
    r_hi = run_recall(hi)
    if r_hi < goal:
        return hi, r_hi
    best = (hi, r_hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        r = run_recall(mid)
        if r >= goal:
            hi = mid
            best = (mid, r)
        else:
            lo = mid
    return best
