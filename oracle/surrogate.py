"""FP64 oracle of the learned support-radius pruning (test infrastructure only).

Used by the test suite, the smoke check and the benchmark's CPU-baseline leg;
never by the product package.

What it defines (the readings are listed in the design notes):
  * labels: per Gaussian, the largest Mahalanobis distance over the HR pixels
    of its exact 3-sigma box whose own contribution alpha max(c) f (Eq. 1, 2)
    is at least tau (``oracle.radius_labels``, plain C);
  * features: [log s, log sigma_x, log sigma_y, rho, alpha, c_r, c_g, c_b]
    (the paper's Gaussian properties of Sec. 3.1 minus the position, plus the
    scale), standardised with training mean / std;
  * a 3-layer MLP 8 -> 64 -> 64 -> 1 (ReLU, ReLU, linear) whose matrix
    products take BF16-rounded operands and accumulate exactly (FP64 here):
    weights, each layer's input activations, and in the backward each layer's
    incoming gradient are rounded to BF16 (round to nearest even) at exactly
    the points where the GPU kernels feed their matrix cores;
  * the pinball (quantile) loss and its gradient;
  * Adam (Kingma & Ba 2015) on FP32 master weights;
  * the pruned radius: min(prediction + margin, 3), or 3 (the exact box) when
    a feature lies outside the training range or the prediction is not finite.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID = 8, 64
PARAM_SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)),
                ("b2", (N_HID,)), ("W3", (1, N_HID)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)  # 4801


def bf16(x):
    """Round to the nearest BF16 value (ties to even); returns FP64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(scale, chol, color, opacity):
    """[N, 8] FP64 features of the Gaussians (scale per Gaussian)."""
    chol = np.asarray(chol, np.float64)
    l11, l21, l22 = chol[:, 0], chol[:, 1], chol[:, 2]
    sx = l11
    sy = np.sqrt(l21 * l21 + l22 * l22)
    rho = l21 / sy
    s = np.broadcast_to(np.asarray(scale, np.float64), l11.shape)
    col = np.asarray(color, np.float64)
    return np.stack([np.log(s), np.log(sx), np.log(sy), rho,
                     np.asarray(opacity, np.float64), col[:, 0], col[:, 1], col[:, 2]], axis=1)


def init_params(seed=0):
    """He-style initialisation, FP32 master weights, flat in PARAM_SHAPES order."""
    rng = np.random.default_rng([seed, 0x5A])
    parts = []
    for name, shape in PARAM_SHAPES:
        if name.startswith("W"):
            fan_in = shape[1]
            parts.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), size=shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


def unpack(flat):
    out, k = {}, 0
    flat = np.asarray(flat)
    for name, shape in PARAM_SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[k:k + n].reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in PARAM_SHAPES])


def mlp_forward(params, X, rounding=True):
    """Prediction [N] for standardised features X [N, 8]; returns (out, cache)."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    p = unpack(params)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    b1, b2, b3 = (np.asarray(p[k], np.float64) for k in ("b1", "b2", "b3"))
    Xb = r(X)
    Z1 = Xb @ W1.T + b1
    H1 = r(np.maximum(Z1, 0.0))
    Z2 = H1 @ W2.T + b2
    H2 = r(np.maximum(Z2, 0.0))
    out = (H2 @ W3.T)[:, 0] + b3[0]
    return out, (Xb, Z1, H1, Z2, H2, W1, W2, W3)


def mlp_backward(cache, dout, rounding=True, parts=None):
    """Flat gradient (PARAM_SHAPES order) for upstream dout [N].  When parts
    is a dict it receives the backward's intermediate values (d3b, dZ2, dZ2b,
    dH1, dZ1, dZ1b), for tests that bound the GPU's rounding against them."""
    r = bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    Xb, Z1, H1, Z2, H2, W1, W2, W3 = cache
    d3 = np.asarray(dout, np.float64)
    d3b = r(d3)
    dW3 = (d3b[None, :] @ H2)
    db3 = np.array([d3.sum()])
    dZ2 = (d3b[:, None] * W3[0][None, :]) * (Z2 > 0)
    dZ2b = r(dZ2)
    dW2 = dZ2b.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2b @ W2) * (Z1 > 0)
    dZ1b = r(dZ1)
    dW1 = dZ1b.T @ Xb
    db1 = dZ1.sum(axis=0)
    if parts is not None:
        parts.update(d3=d3, d3b=d3b, dZ2=dZ2, dZ2b=dZ2b, dH1=dZ2b @ W2, dZ1=dZ1, dZ1b=dZ1b)
    return pack({"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3})


def pinball(pred, label, q):
    """Mean quantile loss of residual u = label - pred and d loss / d pred:
    -q/N where u > 0, (1-q)/N where u <= 0."""
    u = np.asarray(label, np.float64) - np.asarray(pred, np.float64)
    n = u.size
    loss = float(np.where(u > 0, q * u, (q - 1.0) * u).sum() / n)
    grad = np.where(u > 0, -q, 1.0 - q) / n
    return loss, grad


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, exact=False):
    """One Adam step (t counts from 1); returns (params, m, v) in FP32, or
    unrounded in FP64 with exact=True."""
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps)
    if exact:
        return p, m, v
    return p.astype(np.float32), m.astype(np.float32), v.astype(np.float32)


def closed_form_radius(chol, color, opacity, tau, margin=0.0):
    """The support radius without the learned part: the Mahalanobis distance d
    at which alpha max(c) f (Eq. 1, 2) at distance d, alpha max(c) K
    exp(-d^2/2) with K = 1 / (2 pi sigma_x sigma_y sqrt(1 - rho^2)), falls to
    tau; plus margin, clamped to [0, 3]; 3 for invalid values."""
    chol = np.asarray(chol, np.float64)
    sx = chol[:, 0]
    sy = np.sqrt(chol[:, 1] ** 2 + chol[:, 2] ** 2)
    # invalid shapes (l22 = 0 gives |rho| = 1) divide by zero here; they are
    # mapped to 3 below
    with np.errstate(invalid="ignore", divide="ignore"):
        rho = chol[:, 1] / sy
        K = 1.0 / (2.0 * math.pi * sx * sy * np.sqrt(1.0 - rho * rho))
        peak = np.asarray(opacity, np.float64) * np.asarray(color, np.float64).max(axis=1) * K
        d = np.sqrt(2.0 * np.log(np.maximum(peak / tau, 1.0)))
    R = np.clip(d + margin, 0.0, 3.0)
    ok = (chol[:, 0] > 0) & (chol[:, 2] > 0) & np.isfinite(peak)
    return np.where(ok, R, 3.0)


def prune_radius(pred, margin, F, fmin, fmax):
    """Support half-width (in standard deviations) used by the pruned path."""
    pred = np.asarray(pred, np.float64)
    inside = np.all((F >= fmin) & (F <= fmax), axis=1) & np.isfinite(pred)
    R = np.minimum(pred + margin, 3.0)
    return np.where(inside, np.maximum(R, 0.0), 3.0)
