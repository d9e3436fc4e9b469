"""Gaussian primary head and Y-channel PSNR through the C ABI (argument
marshalling only; the arithmetic runs in gs_head.hip).

    mean, chol, color, opacity = gaussian_head(images, grid, raw_opacity,
                                               raw_color, raw_sigma, raw_rho, offset)
    psnr, sse = psnr_y(plan, test, ref, crop=0)

`gaussian_head` is differentiable (`GaussianHead`, a torch.autograd.Function
whose backward is gs_gaussian_head_backward).
"""
from __future__ import annotations

import ctypes
from typing import Sequence, Tuple

import torch

from . import _native as N
from .raster import _ptr, _stream

__all__ = ["GaussianHead", "gaussian_head", "head_images", "psnr_y"]


def head_images(sizes: Sequence[Tuple[int, int]], grid: int):
    """The packed batch layout of images of LR sizes (H, W) with grid^2 H W
    Gaussians each: a list of (lr_h, lr_w, g_begin, g_count)."""
    out, g = [], 0
    for h, w in sizes:
        n = grid * grid * int(h) * int(w)
        out.append((int(h), int(w), g, n))
        g += n
    return out


def _img_array(images):
    arr = (N.gs_image * len(images))()
    for k, (h, w, gb, gc) in enumerate(images):
        arr[k] = N.gs_image(h, w, 1.0, gb, gc, 0)
    return arr


def _check(t, name, shape):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class GaussianHead(torch.autograd.Function):
    @staticmethod
    def forward(ctx, raw_opacity, raw_color, raw_sigma, raw_rho, offset, images, grid):
        n = raw_opacity.shape[0]
        for t, name, sh in ((raw_opacity, "raw_opacity", (n,)), (raw_color, "raw_color", (n, 3)),
                            (raw_sigma, "raw_sigma", (n, 2)), (raw_rho, "raw_rho", (n,)),
                            (offset, "offset", (n, 2))):
            _check(t, name, sh)
        dev = raw_opacity.device
        mean = torch.empty(n, 2, device=dev)
        chol = torch.empty(n, 3, device=dev)
        color = torch.empty(n, 3, device=dev)
        opacity = torch.empty(n, device=dev)
        arr = _img_array(images)
        N.check(N.lib().gs_gaussian_head_forward(
            arr, len(images), int(grid), _ptr(raw_opacity), _ptr(raw_color), _ptr(raw_sigma),
            _ptr(raw_rho), _ptr(offset), n, _ptr(mean), _ptr(chol), _ptr(color),
            _ptr(opacity), _stream()), "gaussian head")
        ctx.save_for_backward(raw_opacity, raw_color, raw_sigma, raw_rho)
        return mean, chol, color, opacity

    @staticmethod
    def backward(ctx, g_mean, g_chol, g_color, g_opacity):
        raw_opacity, raw_color, raw_sigma, raw_rho = ctx.saved_tensors
        n = raw_opacity.shape[0]
        dev = raw_opacity.device

        def grad_or_zero(g, shape):
            return torch.zeros(shape, device=dev) if g is None else g.contiguous()
        g_mean = grad_or_zero(g_mean, (n, 2))
        g_chol = grad_or_zero(g_chol, (n, 3))
        g_color = grad_or_zero(g_color, (n, 3))
        g_opacity = grad_or_zero(g_opacity, (n,))
        d = [torch.empty(s, device=dev) for s in [(n,), (n, 3), (n, 2), (n,), (n, 2)]]
        N.check(N.lib().gs_gaussian_head_backward(
            n, _ptr(raw_opacity), _ptr(raw_color), _ptr(raw_sigma), _ptr(raw_rho),
            _ptr(g_mean), _ptr(g_chol), _ptr(g_color), _ptr(g_opacity), *[_ptr(x) for x in d],
            _stream()), "gaussian head backward")
        return (*d, None, None)


def gaussian_head(images, grid, raw_opacity, raw_color, raw_sigma, raw_rho, offset):
    """(mean, chol, color, opacity) from the five heads' raw outputs.
    images: [(lr_h, lr_w, g_begin, g_count)] (see head_images)."""
    return GaussianHead.apply(raw_opacity, raw_color, raw_sigma, raw_rho, offset,
                              [tuple(int(v) for v in im) for im in images], int(grid))


def psnr_y(plan, test: torch.Tensor, ref: torch.Tensor, crop: int = 0, stream=None):
    """Per-image Y-channel PSNR of two packed outputs of a RasterPlan layout:
    (psnr [n_img] float64, sum of squared Y differences [n_img] float64), on
    the device."""
    _check(test, "test", (plan.out_numel,))
    _check(ref, "ref", (plan.out_numel,))
    n = len(plan.images)
    psnr = torch.empty(n, dtype=torch.float64, device=test.device)
    sse = torch.empty(n, dtype=torch.float64, device=test.device)
    N.check(N.lib().gs_psnr_y(plan._arr, n, _ptr(test), _ptr(ref), int(crop), _ptr(sse),
                              _ptr(psnr), _stream(stream)), "psnr y")
    return psnr, sse
