"""Seeded synthetic workloads for the scale-aware 2D Gaussian rasterizer.

This module only draws inputs; it holds none of the rasterizer's arithmetic.
Both the HIP path (tests, benchmark, smoke check) and the FP64 oracle are fed
from here.  Every draw comes from ``numpy.random.default_rng([seed, k])`` for
image k, in FP64, and is then cast to FP32; the FP32 arrays are the canonical
inputs.

Shapes follow the paper's setting: one Gaussian per LR pixel placed on the LR
grid (the paper's reference positions sit at equal intervals over the LR
image, Sec. 3.2, and the position is reference plus a free offset), LR pixel
centres at integer coordinates (Eq. 3 samples integer x in [0, W-1]).  The
covariance is handed over as its Cholesky factor (l11, l21, l22) of
Sigma = R(theta) diag(s1^2, s2^2) R(theta)^T.

Workloads (HR size = floor(s*LR + 0.5)):
  tiny     : parity cases, a few Gaussians on a small image.
  config0  : 48x48 LR, 2,304 Gaussians, s = 4 -> 192x192, forward only.
  config1  : 16 images of 64x64 LR, 4,096 Gaussians each, s = 3.7 -> 237x237,
             L1 loss to a seeded uniform target.
  config2a : 512x512 LR, 262,144 Gaussians, s = 4 -> 2048x2048, wide sigmas.
  config2b : 256x256 LR, 65,536 Gaussians, s = 12 -> 3072x3072, wide sigmas.
  config3  : 64 images, H, W ~ U{48..256}, 25% extra Gaussians at uniform
             random positions, s ~ U[1.5, 12].
  paper720 : the paper's cost workload: a 720x720 HR output at s in
             {2, 3, 4, 6, 8, 12} from a (720/s)^2 LR image holding m = 16
             Gaussians per LR pixel, one per cell of a 4x4 sub-grid of each
             pixel with a free offset inside its cell; per-axis log-std
             N(log 0.35, 0.3) LR pixels (not published: a stand-in).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Image", "Workload", "draw_image_gaussians", "cholesky_from_axes",
    "tiny", "config0", "config1", "config2a", "config2b", "config3",
    "paper720", "draw_grid_gaussians", "by_name", "concat",
]


@dataclasses.dataclass
class Image:
    lr_h: int
    lr_w: int
    scale: float
    g_begin: int
    g_count: int


@dataclasses.dataclass
class Workload:
    """A batch of images whose Gaussians are packed image after image."""
    name: str
    images: List[Image]
    mean: np.ndarray      # [N, 2] float32 (mu_x, mu_y) in LR pixels
    chol: np.ndarray      # [N, 3] float32 (l11, l21, l22)
    color: np.ndarray     # [N, 3] float32
    opacity: np.ndarray   # [N]    float32
    target: Optional[np.ndarray] = None   # list-like per image, or None

    @property
    def n_gauss(self) -> int:
        return int(self.mean.shape[0])

    def image_slice(self, k: int) -> slice:
        im = self.images[k]
        return slice(im.g_begin, im.g_begin + im.g_count)


def cholesky_from_axes(s1: np.ndarray, s2: np.ndarray, theta: np.ndarray):
    """Cholesky factor of R(theta) diag(s1^2, s2^2) R(theta)^T, in FP64.

    l11 = sqrt(Sxx), l21 = Sxy / l11, l22 = sqrt(det) / l11 = s1 s2 / l11.
    """
    c, s = np.cos(theta), np.sin(theta)
    sxx = c * c * s1 * s1 + s * s * s2 * s2
    sxy = c * s * (s1 * s1 - s2 * s2)
    l11 = np.sqrt(sxx)
    l21 = sxy / l11
    l22 = s1 * s2 / l11
    return l11, l21, l22


def draw_image_gaussians(rng: np.random.Generator, H: int, W: int,
                         log_sigma_mean: float, log_sigma_std: float,
                         extra_frac: float = 0.0):
    """One Gaussian per LR pixel (row-major) with U[-1/2, 1/2]^2 jitter, plus
    round(extra_frac * H * W) Gaussians uniformly placed over the image.

    Returns FP32 arrays (mean [N,2], chol [N,3], color [N,3], opacity [N]).
    """
    n_grid = H * W
    n_extra = int(round(extra_frac * n_grid))
    n = n_grid + n_extra
    jy, jx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                         indexing="ij")
    mean = np.empty((n, 2), dtype=np.float64)
    mean[:n_grid, 0] = jx.ravel()
    mean[:n_grid, 1] = jy.ravel()
    mean[:n_grid] += rng.uniform(-0.5, 0.5, size=(n_grid, 2))
    if n_extra:
        mean[n_grid:, 0] = rng.uniform(-0.5, W - 0.5, size=n_extra)
        mean[n_grid:, 1] = rng.uniform(-0.5, H - 0.5, size=n_extra)
    log_sig = rng.normal(math.log(log_sigma_mean), log_sigma_std, size=(n, 2))
    theta = rng.uniform(0.0, math.pi, size=n)
    color = rng.uniform(0.0, 1.0, size=(n, 3))
    opacity = rng.uniform(0.5, 1.0, size=n)
    l11, l21, l22 = cholesky_from_axes(np.exp(log_sig[:, 0]), np.exp(log_sig[:, 1]), theta)
    chol = np.stack([l11, l21, l22], axis=1)
    return (mean.astype(np.float32), chol.astype(np.float32),
            color.astype(np.float32), opacity.astype(np.float32))


def draw_grid_gaussians(rng: np.random.Generator, H: int, W: int, grid: int,
                        log_sigma_mean: float, log_sigma_std: float):
    """grid^2 Gaussians per LR pixel, row-major over a (grid H) x (grid W)
    sub-grid of equal cells covering [-1/2, W - 1/2] x [-1/2, H - 1/2], each
    uniformly inside its own cell.  FP32 (mean, chol, color, opacity)."""
    gx = (np.arange(grid * W, dtype=np.float64) + 0.5) / grid - 0.5
    gy = (np.arange(grid * H, dtype=np.float64) + 0.5) / grid - 0.5
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    n = X.size
    mean = np.stack([X.ravel(), Y.ravel()], axis=1)
    mean += rng.uniform(-0.5 / grid, 0.5 / grid, size=(n, 2))
    log_sig = rng.normal(math.log(log_sigma_mean), log_sigma_std, size=(n, 2))
    theta = rng.uniform(0.0, math.pi, size=n)
    color = rng.uniform(0.0, 1.0, size=(n, 3))
    opacity = rng.uniform(0.5, 1.0, size=n)
    l11, l21, l22 = cholesky_from_axes(np.exp(log_sig[:, 0]), np.exp(log_sig[:, 1]), theta)
    chol = np.stack([l11, l21, l22], axis=1)
    return (mean.astype(np.float32), chol.astype(np.float32),
            color.astype(np.float32), opacity.astype(np.float32))


def paper720(s: int = 4, seed: int = 0, with_target: bool = False, hr: int = 720,
             grid: int = 4) -> "Workload":
    """The paper's rendering-cost workload at integer scale s: an hr x hr
    output (720 by default) from an (hr/s)^2 LR image with grid^2 Gaussians
    per LR pixel (m = 16)."""
    if hr % s:
        raise ValueError("the HR side must be a multiple of the scale")
    H = W = hr // s
    rng = np.random.default_rng([seed, 0])
    m, c, col, op = draw_grid_gaussians(rng, H, W, grid, 0.35, 0.3)
    targets = None
    if with_target:
        targets = [np.random.default_rng([seed, 0, 1]).uniform(0.0, 1.0, size=(3, hr, hr))
                   .astype(np.float32)]
    return Workload(name=f"paper720_x{s}", images=[Image(H, W, float(s), 0, m.shape[0])],
                    mean=m, chol=c, color=col, opacity=op, target=targets)


def _build(name, shapes, sigma, extra_frac, seed, with_target=False):
    parts = []
    images = []
    begin = 0
    targets = [] if with_target else None
    for k, (H, W, s) in enumerate(shapes):
        rng = np.random.default_rng([seed, k])
        m, c, col, op = draw_image_gaussians(rng, H, W, sigma[0], sigma[1], extra_frac)
        parts.append((m, c, col, op))
        images.append(Image(H, W, float(s), begin, m.shape[0]))
        begin += m.shape[0]
        if with_target:
            oh = int(math.floor(s * H + 0.5))
            ow = int(math.floor(s * W + 0.5))
            trng = np.random.default_rng([seed, k, 1])
            targets.append(trng.uniform(0.0, 1.0, size=(3, oh, ow)).astype(np.float32))
    return Workload(
        name=name, images=images,
        mean=np.concatenate([p[0] for p in parts]),
        chol=np.concatenate([p[1] for p in parts]),
        color=np.concatenate([p[2] for p in parts]),
        opacity=np.concatenate([p[3] for p in parts]),
        target=targets,
    )


def tiny(H=5, W=6, s=2.5, seed=0, sigma=(0.6, 0.3), extra_frac=0.0, n_images=1,
         with_target=False):
    """Small parity case (default 30 Gaussians)."""
    return _build(f"tiny{H}x{W}s{s}", [(H, W, s)] * n_images, sigma, extra_frac, seed,
                  with_target)


def config0(seed=0, with_target=False):
    """48x48 LR, one Gaussian per LR pixel, x4 -> 192x192 (forward parity case)."""
    return _build("c0_48x48_s4", [(48, 48, 4.0)], (0.6, 0.3), 0.0, seed, with_target)


def config1(seed=0, n_images=16):
    """16 x (64x64 LR, 4,096 Gaussians) at x3.7 -> 237x237, L1 to a uniform target."""
    return _build("c1_16x64x64_s3.7", [(64, 64, 3.7)] * n_images, (0.6, 0.3), 0.0, seed,
                  with_target=True)


def config2a(seed=0):
    """512x512 LR (262,144 Gaussians) at x4 -> 2048x2048; log-std N(log 0.8, 0.5)."""
    return _build("c2a_512x512_s4", [(512, 512, 4.0)], (0.8, 0.5), 0.0, seed, with_target=True)


def config2b(seed=0):
    """256x256 LR (65,536 Gaussians) at x12 -> 3072x3072; log-std N(log 0.8, 0.5)."""
    return _build("c2b_256x256_s12", [(256, 256, 12.0)], (0.8, 0.5), 0.0, seed,
                  with_target=True)


def config3_shapes(seed=0, n_images=64):
    """Uneven batch: H, W ~ U{48..256} independently, s ~ U[1.5, 12]."""
    rng = np.random.default_rng([seed, 0xC3])
    H = rng.integers(48, 257, size=n_images)
    W = rng.integers(48, 257, size=n_images)
    s = rng.uniform(1.5, 12.0, size=n_images)
    return [(int(h), int(w), float(sc)) for h, w, sc in zip(H, W, s)]


def config3(seed=0, n_images=64, with_target=False):
    """64 uneven images, one Gaussian per LR pixel plus 25% extra."""
    return _build("c3_64uneven", config3_shapes(seed, n_images), (0.6, 0.3), 0.25, seed,
                  with_target)


def by_name(name: str, seed: int = 0, with_target: bool = False) -> Workload:
    """The named workload; with_target adds the L1 targets to the ones that
    are built without (config0, config3)."""
    if name in ("config0", "config3"):
        return {"config0": config0, "config3": config3}[name](seed=seed, with_target=with_target)
    return {"config1": config1, "config2a": config2a, "config2b": config2b}[name](seed=seed)


def concat(workloads: List[Workload], name="concat") -> Workload:
    """Pack several workloads into one batch."""
    images, begin = [], 0
    for w in workloads:
        for im in w.images:
            images.append(Image(im.lr_h, im.lr_w, im.scale, begin, im.g_count))
            begin += im.g_count
    tg = None
    if all(w.target is not None for w in workloads):
        tg = [t for w in workloads for t in w.target]
    return Workload(name, images,
                    np.concatenate([w.mean for w in workloads]),
                    np.concatenate([w.chol for w in workloads]),
                    np.concatenate([w.color for w in workloads]),
                    np.concatenate([w.opacity for w in workloads]), tg)


def surrogate_training_batch(seed: int, k: int, n_images: int = 16, lr_side: int = 24):
    """Training batch k for the learned support radius: n_images LR
    lr_side x lr_side images, one Gaussian per LR pixel plus 25% extra, with
    the per-axis log-std of config 2 (even k) or of configs 0/1/3 (odd k),
    and scales U[1.4, 12.6] (slightly wider than the workloads' [1.5, 12]).

    Returns (images, mean, chol, color, opacity), images as
    (lr_h, lr_w, scale, g_begin, g_count)."""
    rng = np.random.default_rng([seed, k, 7])
    sig = (0.8, 0.5) if k % 2 == 0 else (0.6, 0.3)
    parts, images, begin = [], [], 0
    for j in range(n_images):
        s = float(rng.uniform(1.4, 12.6))
        g = draw_image_gaussians(np.random.default_rng([seed, k, j]), lr_side, lr_side,
                                 sig[0], sig[1], 0.25)
        parts.append(g)
        images.append((lr_side, lr_side, s, begin, g[0].shape[0]))
        begin += g[0].shape[0]
    return (images,) + tuple(np.concatenate([p[i] for p in parts]) for i in range(4))
