"""FP64 oracle of the Gaussian primary head and of the Y-channel PSNR
(test infrastructure only: imported by the test suite, never by the product
package).

Gaussian primary head (Sec. 3.2, "Gaussian Primary Head" and "Gaussian
Embedding").  Five heads give, per Gaussian, raw outputs for the opacity,
the colour, the standard deviations, the reference offset and the
correlation.  The properties of Sec. 3.1 follow from them:
  * alpha = sigmoid(a), c = sigmoid(r) (per channel), sigma = sigmoid(u)
    (per axis), rho = tanh(v), and no activation on the offset o;
  * mu = p + o, with p the Gaussian's reference position: N = m H W points
    taken at equal intervals over the H x W LR image (m = g^2 points per LR
    pixel, g per axis), read here as the centres of a (g H) x (g W) grid of
    equal cells over the image area [-1/2, W - 1/2] x [-1/2, H - 1/2] (LR
    pixel centres at integers), numbered row-major;
  * the rasterizer takes the covariance of Eq. 2 as its Cholesky factor:
    l11 = sigma_x, l21 = rho sigma_y, l22 = sigma_y sqrt(1 - rho^2), so
    L L^T = [[sigma_x^2, rho sigma_x sigma_y], [rho sigma_x sigma_y, sigma_y^2]].
The backward is the chain rule through these definitions.

Y-channel PSNR (Sec. 4.1, evaluation protocols: PSNR on the Y channel of
YCbCr).  Y is the ITU-R BT.601 luma in studio range, the usual convention of
super-resolution evaluation, for RGB on [0, 1]:
    Y = (16 + 65.481 R + 128.553 G + 24.966 B) / 255,
and PSNR = 10 log10(1 / MSE) of Y over the image, optionally without a
border of `crop` pixels; no clamping or quantisation.
"""
from __future__ import annotations

import math

import numpy as np

Y_COEF = (65.481, 128.553, 24.966)
Y_OFFSET = 16.0


def reference_positions(H, W, grid):
    """[grid^2 H W, 2] reference positions (x, y) of one LR image, row-major
    over the (grid H) x (grid W) grid of cell centres."""
    px = (np.arange(grid * W, dtype=np.float64) + 0.5) / grid - 0.5
    py = (np.arange(grid * H, dtype=np.float64) + 0.5) / grid - 0.5
    X, Y = np.meshgrid(px, py, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def _sigmoid(x):
    x = np.asarray(x, np.float64)
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-x))


def head_forward(raw_opacity, raw_color, raw_sigma, raw_rho, offset, ref_pos):
    """(mean [N,2], chol [N,3], color [N,3], opacity [N]) from the heads' raw
    outputs and the reference positions."""
    alpha = _sigmoid(raw_opacity)
    color = _sigmoid(raw_color)
    sigma = _sigmoid(raw_sigma)
    rho = np.tanh(np.asarray(raw_rho, np.float64))
    mean = np.asarray(ref_pos, np.float64) + np.asarray(offset, np.float64)
    sx, sy = sigma[:, 0], sigma[:, 1]
    chol = np.stack([sx, rho * sy, sy * np.sqrt(1.0 - rho * rho)], axis=1)
    return mean, chol, color, alpha


def head_backward(raw_opacity, raw_color, raw_sigma, raw_rho, g_mean, g_chol, g_color,
                  g_opacity):
    """Gradients w.r.t. (raw_opacity [N], raw_color [N,3], raw_sigma [N,2],
    raw_rho [N], offset [N,2]) from those w.r.t. the head's outputs.  The
    sigmoid's derivative s(x) (1 - s(x)) is taken as s(x) s(-x), the same
    number without the cancellation of 1 - s(x)."""
    a = np.asarray(raw_opacity, np.float64)
    r = np.asarray(raw_color, np.float64)
    u = np.asarray(raw_sigma, np.float64)
    v = np.asarray(raw_rho, np.float64)
    g_chol = np.asarray(g_chol, np.float64)
    d_opacity = np.asarray(g_opacity, np.float64) * _sigmoid(a) * _sigmoid(-a)
    d_color = np.asarray(g_color, np.float64) * _sigmoid(r) * _sigmoid(-r)
    sigma = _sigmoid(u)
    sx, sy = sigma[:, 0], sigma[:, 1]
    rho = np.tanh(v)
    root = np.sqrt(1.0 - rho * rho)
    g11, g21, g22 = g_chol[:, 0], g_chol[:, 1], g_chol[:, 2]
    dL_dsx = g11
    dL_dsy = g21 * rho + g22 * root
    dL_drho = g21 * sy - g22 * sy * rho / root
    d_sigma = np.stack([dL_dsx, dL_dsy], axis=1) * sigma * _sigmoid(-u)
    d_rho = dL_drho * (1.0 - rho * rho)
    d_offset = np.asarray(g_mean, np.float64).copy()
    return d_opacity, d_color, d_sigma, d_rho, d_offset


def rgb_to_y(img):
    """BT.601 studio-range luma of a planar [3, h, w] RGB image on [0, 1]."""
    img = np.asarray(img, np.float64)
    return (Y_OFFSET + Y_COEF[0] * img[0] + Y_COEF[1] * img[1] + Y_COEF[2] * img[2]) / 255.0


def psnr_y(test, ref, crop=0):
    """(PSNR in dB, sum of squared Y differences, pixel count) of one planar
    [3, h, w] image against a reference, without a border of crop pixels."""
    yt, yr = rgb_to_y(test), rgb_to_y(ref)
    h, w = yt.shape
    yt = yt[crop:h - crop, crop:w - crop]
    yr = yr[crop:h - crop, crop:w - crop]
    d = yt - yr
    sse = float((d * d).sum())
    n = d.size
    if n == 0:
        return math.nan, 0.0, 0
    mse = sse / n
    return (math.inf if mse == 0.0 else 10.0 * math.log10(1.0 / mse)), sse, n
