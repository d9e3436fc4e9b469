"""Training and calibration of the learned support radius (orchestration only).

Every numeric step on the data is a library kernel: the exact rasterizer
bins each batch and measures the labels, the feature kernel standardises,
the MLP gradient and Adam kernels train, the MLP forward kernel predicts.
The host only picks batches and keeps dataset-level statistics (feature mean
and spread, the training range, and the quantile of the held-out residuals
that becomes the margin).

A batch comes from a caller-supplied function ``make_batch(k)`` returning
(images, mean, chol, color, opacity) with images a list of
(lr_h, lr_w, scale, g_begin, g_count) and FP32 numpy arrays.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List

import numpy as np
import torch

from .raster import RasterPlan
from .surrogate import RadiusMLP, features, make_norm, radius_labels


@dataclasses.dataclass
class Batch:
    feats: torch.Tensor    # features [n, 8] (standardised unless noted)
    labels: torch.Tensor   # [n]


def make_batches(make_batch: Callable, ks, tau: float, norm=None, device="cuda",
                 tile: int = 16, with_labels=True) -> List[Batch]:
    """Features (standardised with norm, raw without) and, optionally, labels
    measured by the exact rasterizer, for the Gaussians of batches ks whose
    support box the image border does not cut (their labels are whole)."""
    out = []
    for k in ks:
        images, mean, chol, color, opacity = make_batch(k)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        m, c, col, op = t(mean), t(chol), t(color), t(opacity)
        plan = RasterPlan(images, mean.shape[0], tile=tile)
        F = features(plan, c, col, op, norm)
        plan.ensure_capacity(m, c)
        ws = plan.new_workspace(device)
        plan.bin(m, c, col, op, ws)
        lab = radius_labels(plan, ws, tau, interior_only=True)
        idx = torch.nonzero(lab >= 0).flatten()
        out.append(Batch(F.index_select(0, idx).contiguous(),
                         lab.index_select(0, idx).contiguous() if with_labels else None))
    return out


def init_params(seed=0):
    """He initialisation of the weights, zero hidden biases, output bias 1.5
    (the middle of the label range); FP32, flat layout."""
    rng = np.random.default_rng([seed, 0x5A])
    W1 = rng.normal(0.0, math.sqrt(2.0 / 8), size=(64, 8))
    W2 = rng.normal(0.0, math.sqrt(2.0 / 64), size=(64, 64))
    W3 = rng.normal(0.0, math.sqrt(2.0 / 64), size=(1, 64))
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3.ravel(),
                           [1.5]]).astype(np.float32)


def train_radius_mlp(make_batch: Callable, n_train: int, n_calib: int, tau: float,
                     steps: int = 400, lr: float = 2e-3, quantile: float = 0.9,
                     coverage: float = 0.999, n_stats: int = 8, device="cuda", log=None):
    """Dataset from the exact rasterizer, training, margin calibration.

    Batches 0 .. n_train-1 train, the next n_calib calibrate.  Returns
    (net, info) with net.norm holding the standardisation, the training range
    of the standardised features and the margin (the `coverage` quantile of
    label - prediction on the held-out batches)."""
    t0 = time.perf_counter()
    raw = make_batches(make_batch, range(min(n_stats, n_train)), tau, None, device,
                       with_labels=False)
    R = np.concatenate([b.feats.cpu().numpy().astype(np.float64) for b in raw])
    mu, sd = R.mean(0), R.std(0)
    sd[sd == 0] = 1.0
    norm0 = make_norm(mu, sd)
    train = make_batches(make_batch, range(n_train), tau, norm0, device)
    calib = make_batches(make_batch, range(n_train, n_train + n_calib), tau, norm0, device)
    Z = np.concatenate([b.feats.cpu().numpy() for b in train])
    fmin, fmax = Z.min(0), Z.max(0)
    t_data = time.perf_counter() - t0

    net = RadiusMLP(init_params(), device)
    rng = np.random.default_rng(1234)
    loss = torch.zeros((), dtype=torch.float64, device=device)
    losses = []
    t1 = time.perf_counter()
    for s in range(steps):
        b = train[int(rng.integers(0, len(train)))]
        loss.zero_()
        net.step(b.feats, b.labels, lr=lr, quantile=quantile, loss=loss)
        if s % 50 == 0 or s == steps - 1:
            losses.append(float(loss.item()))
            if log:
                log(f"surrogate step {s}: pinball loss {losses[-1]:.5f}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    res = np.concatenate([(b.labels - net.predict(b.feats)).cpu().numpy() for b in calib])
    margin = float(max(0.0, np.quantile(res, coverage)))
    net.norm = make_norm(mu, sd, fmin, fmax, margin)
    info = {"train_rows": int(sum(b.labels.numel() for b in train)), "calib_rows": int(res.size),
            "margin": margin, "losses": losses, "seconds_data": round(t_data, 2),
            "seconds_train": round(t_train, 2), "tau": tau, "quantile": quantile,
            "coverage": coverage, "steps": steps}
    return net, info
