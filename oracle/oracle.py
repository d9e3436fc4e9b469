"""Python face of the FP64 CPU oracle (test infrastructure only).

Wraps ``gs_oracle.c`` through ctypes.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg use it; the product path never does.
Inputs are widened from FP32 to FP64 exactly; every result is FP64.

Per-image functions follow the paper directly (see gs_oracle.c for the
passages); the batch helpers only loop over images and lay results out the
way the HIP library does (planar RGB images packed one after another, tile ids
numbered image after image, Gaussian ids global over the packed batch).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libgsoracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no FMA contraction; OpenMP
    for the multi-threaded timing variants only)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_output_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                     _I32, _I32]
        L.or_output_size.restype = ctypes.c_int
        L.or_support_rect.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_int32] + \
            [ctypes.c_double] * 6 + [_I32]
        L.or_support_rect.restype = ctypes.c_int
        L.or_box_cut.argtypes = L.or_support_rect.argtypes[:-1]
        L.or_box_cut.restype = ctypes.c_int
        L.or_forward.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                 ctypes.c_int64, _D, _D, _D, _D, _D, ctypes.c_double,
                                 ctypes.c_int32, _D]
        L.or_forward.restype = None
        L.or_backward.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_int64, _D, _D, _D, _D, _D, ctypes.c_double,
                                  ctypes.c_int32, _D, _D, _D, _D, _D]
        L.or_backward.restype = None
        L.or_forward_mt.argtypes = L.or_forward.argtypes + [ctypes.c_int32]
        L.or_forward_mt.restype = None
        L.or_backward_mt.argtypes = L.or_backward.argtypes + [ctypes.c_int32]
        L.or_backward_mt.restype = None
        L.or_tile_lists.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                    ctypes.c_int64, _D, _D, _D, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32,
                                    ctypes.c_int32, _I32, _I32, ctypes.c_int64]
        L.or_tile_lists.restype = ctypes.c_int64
        L.or_support_pairs.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                       ctypes.c_int32, _I32]
        L.or_support_pairs.restype = ctypes.c_int64
        L.or_pixel_values.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_int64, _D, _D, _D, _D, _D, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_int64,
                                      _I32, _I32, _D]
        L.or_pixel_values.restype = None
        L.or_radius_labels.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, _D]
        L.or_radius_labels.restype = None
        L.or_window_rect.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_double] + \
            [ctypes.c_double] * 5 + [ctypes.c_int32, _I32]
        L.or_support_rect_m.argtypes = [ctypes.c_double, ctypes.c_int32, ctypes.c_int32] + \
            [ctypes.c_double] * 6 + [ctypes.c_int32, _I32]
        L.or_support_rect_m.restype = ctypes.c_int
        L.or_pixel_d2.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_int32] + [ctypes.c_double] * 5
        L.or_pixel_d2.restype = ctypes.c_double
        L.or_window_rect.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    """Exact FP64 widening, C-contiguous."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t=_D):
    return None if a is None else a.ctypes.data_as(t)


# ---------------------------------------------------------------- per image

def output_size(H: int, W: int, s: float):
    oh, ow = ctypes.c_int32(), ctypes.c_int32()
    if lib().or_output_size(H, W, float(s), ctypes.byref(oh), ctypes.byref(ow)) != 0:
        raise ValueError("invalid size")
    return oh.value, ow.value


def support_rect(s, out_w, out_h, mx, my, l11, l21, l22, R=3.0):
    r = (ctypes.c_int32 * 4)()
    ok = lib().or_support_rect(float(s), out_w, out_h, float(mx), float(my), float(l11),
                               float(l21), float(l22), float(R), r)
    return bool(ok), tuple(r)


def box_cut(H, W, s, mean, chol, R=3.0):
    """Per Gaussian: 1 if the image border cuts its support box, 0 if not,
    -1 if it is invalid."""
    oh, ow = output_size(H, W, s)
    mean, chol = _d(mean), _d(chol)
    return np.array([lib().or_box_cut(float(s), ow, oh, *mean[i], *chol[i], float(R))
                     for i in range(mean.shape[0])], dtype=np.int32)


# support-mode bits (see gs_oracle.c): pixel-centre sampling, elliptical support
PIXEL_CENTER = 1
ELLIPSE = 2


def window_rect(s, out_w, out_h, H, W, r, mx, my, l11, l21, l22, mode=0):
    """Algorithm 1's r-window of one Gaussian (see gs_oracle.c)."""
    rr = (ctypes.c_int32 * 4)()
    ok = lib().or_window_rect(float(s), out_w, out_h, H, W, float(r), float(mx), float(my),
                              float(l11), float(l21), float(l22), int(mode), rr)
    return bool(ok), tuple(rr)


def support_rect_m(s, out_w, out_h, mx, my, l11, l21, l22, R=3.0, mode=0):
    """The box of one Gaussian under either sampling convention."""
    r = (ctypes.c_int32 * 4)()
    ok = lib().or_support_rect_m(float(s), out_w, out_h, float(mx), float(my), float(l11),
                                 float(l21), float(l22), float(R), int(mode), r)
    return bool(ok), tuple(r)


def pixel_d2(x, y, s, mode, mx, my, l11, l21, l22):
    """Squared Mahalanobis distance of HR pixel (x, y) (the pinned sequence)."""
    return lib().or_pixel_d2(int(x), int(y), float(s), int(mode), float(mx), float(my),
                             float(l11), float(l21), float(l22))


def support_rects(H, W, s, mean, chol, radius=None, window=0.0, mode=0):
    """Support boxes [n][4] (x0, x1, y0, y1; empty = x1 < x0) and the number of
    in-support (pixel, Gaussian) pairs.  window > 0: Algorithm 1's r-window
    with r = window instead of the standard-deviation box."""
    mean, chol = _d(mean), _d(chol)
    rad = None if radius is None else _d(radius)
    n = mean.shape[0]
    rects = np.zeros((n, 4), dtype=np.int32)
    total = lib().or_support_pairs(H, W, float(s), n, _p(mean), _p(chol), _p(rad),
                                   float(window), int(mode), _p(rects, _I32))
    return rects, int(total)


def forward(H, W, s, mean, chol, color, opacity, radius=None, threads=1, window=0.0, mode=0):
    """HR image [3, out_h, out_w] (FP64) of one image.  threads > 1 runs the
    OpenMP variant (row bands; bitwise the same image)."""
    oh, ow = output_size(H, W, s)
    mean, chol, color, opacity = _d(mean), _d(chol), _d(color), _d(opacity)
    rad = None if radius is None else _d(radius)
    out = np.zeros((3, oh, ow), dtype=np.float64)
    args = (H, W, float(s), mean.shape[0], _p(mean), _p(chol), _p(color), _p(opacity),
            _p(rad), float(window), int(mode), _p(out))
    if threads > 1:
        lib().or_forward_mt(*args, int(threads))
    else:
        lib().or_forward(*args)
    return out


def backward(H, W, s, mean, chol, color, opacity, grad_out, radius=None, threads=1,
             window=0.0, mode=0):
    """Gradients (mean, chol, color, opacity) for upstream dL/dI grad_out.
    threads > 1 runs the OpenMP variant (bitwise the same result)."""
    mean, chol, color, opacity = _d(mean), _d(chol), _d(color), _d(opacity)
    rad = None if radius is None else _d(radius)
    g = _d(grad_out)
    n = mean.shape[0]
    gm, gc = np.zeros((n, 2)), np.zeros((n, 3))
    gcol, gop = np.zeros((n, 3)), np.zeros(n)
    args = (H, W, float(s), n, _p(mean), _p(chol), _p(color), _p(opacity), _p(rad),
            float(window), int(mode), _p(g), _p(gm), _p(gc), _p(gcol), _p(gop))
    if threads > 1:
        lib().or_backward_mt(*args, int(threads))
    else:
        lib().or_backward(*args)
    return gm, gc, gcol, gop


def pixel_values(H, W, s, mean, chol, color, opacity, xs, ys, radius=None, window=0.0,
                 mode=0):
    """Image values [3, npix] at HR pixels (xs[k], ys[k]) of one image."""
    mean, chol, color, opacity = _d(mean), _d(chol), _d(color), _d(opacity)
    rad = None if radius is None else _d(radius)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    out = np.zeros((3, xs.size), dtype=np.float64)
    lib().or_pixel_values(H, W, float(s), mean.shape[0], _p(mean), _p(chol), _p(color),
                          _p(opacity), _p(rad), float(window), int(mode), xs.size, _p(xs, _I32),
                          _p(ys, _I32), _p(out))
    return out


def radius_labels(H, W, s, mean, chol, color, opacity, tau):
    """Per-Gaussian support-radius labels of one image (see gs_oracle.c)."""
    mean, chol, color, opacity = _d(mean), _d(chol), _d(color), _d(opacity)
    R = np.zeros(mean.shape[0])
    lib().or_radius_labels(H, W, float(s), mean.shape[0], _p(mean), _p(chol), _p(color),
                           _p(opacity), float(tau), _p(R))
    return R


def interior_labels_batch(wl, tau):
    """radius_labels_batch with -1 for the Gaussians whose support box the
    image border cuts (or that are invalid)."""
    out = radius_labels_batch(wl, tau)
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        cut = box_cut(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl])
        out[sl] = np.where(cut != 0, -1.0, out[sl])
    return out


def radius_labels_batch(wl, tau):
    out = np.zeros(wl.n_gauss)
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        out[sl] = radius_labels(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl],
                                wl.color[sl], wl.opacity[sl], tau)
    return out


def tile_lists(H, W, s, mean, chol, tw, th, radius=None, window=0.0, mode=0):
    """(counts [tiles] int32, lists [P] int32) for one image."""
    mean, chol = _d(mean), _d(chol)
    rad = None if radius is None else _d(radius)
    oh, ow = output_size(H, W, s)
    n_tiles = ((ow + tw - 1) // tw) * ((oh + th - 1) // th)
    counts = np.zeros(n_tiles, dtype=np.int32)
    total = lib().or_tile_lists(H, W, float(s), mean.shape[0], _p(mean), _p(chol), _p(rad),
                                float(window), int(mode), tw, th, _p(counts, _I32), None, 0)
    lists = np.zeros(max(total, 1), dtype=np.int32)
    total2 = lib().or_tile_lists(H, W, float(s), mean.shape[0], _p(mean), _p(chol), _p(rad),
                                 float(window), int(mode), tw, th, _p(counts, _I32),
                                 _p(lists, _I32), total)
    assert total2 == total
    return counts, lists[:total]


# ----------------------------------------------------------- batch helpers

def _radius_slice(radius, sl):
    return None if radius is None else np.asarray(radius)[sl]


def forward_batch(wl, radius=None, threads=1, window=0.0, mode=0):
    """List of FP64 images [3, oh, ow], one per image of the workload."""
    out = []
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        out.append(forward(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl],
                           wl.color[sl], wl.opacity[sl], _radius_slice(radius, sl), threads,
                           window, mode))
    return out


def backward_batch(wl, grads_out, radius=None, threads=1, window=0.0, mode=0):
    """Packed gradients over the whole batch for per-image upstream gradients."""
    n = wl.n_gauss
    gm, gc = np.zeros((n, 2)), np.zeros((n, 3))
    gcol, gop = np.zeros((n, 3)), np.zeros(n)
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        a, b, c, d = backward(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl],
                              wl.color[sl], wl.opacity[sl], grads_out[k],
                              _radius_slice(radius, sl), threads, window, mode)
        gm[sl], gc[sl], gcol[sl], gop[sl] = a, b, c, d
    return gm, gc, gcol, gop


def tile_lists_batch(wl, tw, th, radius=None, window=0.0, mode=0):
    """Tile ranges and concatenated lists with tiles numbered image after image
    and Gaussian ids global over the packed batch.

    Returns (ranges [tiles, 2] int32 as [begin, end) into lists, lists int32).
    Empty tiles get [0, 0)."""
    counts_all, lists_all = [], []
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        c, l = tile_lists(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl], tw, th,
                          _radius_slice(radius, sl), window, mode)
        counts_all.append(c)
        lists_all.append(l + im.g_begin)
    counts = np.concatenate(counts_all).astype(np.int64)
    lists = np.concatenate(lists_all).astype(np.int32) if lists_all else np.zeros(0, np.int32)
    ends = np.cumsum(counts)
    begins = ends - counts
    ranges = np.stack([begins, ends], axis=1)
    ranges[counts == 0] = 0
    return ranges.astype(np.int32), lists


def support_pairs_batch(wl, radius=None, window=0.0, mode=0):
    """Total in-support (pixel, Gaussian) pairs over the batch."""
    total = 0
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        total += support_rects(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl],
                               _radius_slice(radius, sl), window, mode)[1]
    return total


def l1_loss_and_grad(images, targets):
    """Mean absolute error over every element of the batch and its gradient
    sign(I - T) / numel (sign(0) = 0), the training loss of Sec. 3.2 ("Rendering")."""
    numel = sum(int(np.asarray(t).size) for t in targets)
    loss = 0.0
    grads = []
    for I, T in zip(images, targets):
        d = np.asarray(I, np.float64) - np.asarray(T, np.float64)
        loss += float(np.abs(d).sum())
        grads.append(np.sign(d) / numel)
    return loss / numel, grads


def psnr(test, ref, peak=1.0):
    """10 log10(peak^2 / MSE) over every value of the batch (no clamping)."""
    se, n = 0.0, 0
    for a, b in zip(test, ref):
        d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
        se += float((d * d).sum())
        n += d.size
    mse = se / n
    return math.inf if mse == 0.0 else 10.0 * math.log10(peak * peak / mse)
