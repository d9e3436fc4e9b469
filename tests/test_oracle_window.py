"""Pins of the oracle's r-window support (Algorithm 1's rasterization ratio,
Sec. 3.1 "Fast Rasterization") against exact arithmetic, brute force and the
untruncated render the window converges to."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import synth
from oracle import oracle as O


def _out_size(H, W, s):
    return int(math.floor(s * H + 0.5)), int(math.floor(s * W + 0.5))


def brute_force_window(H, W, s, r, mean, chol, color, opacity):
    """Every Gaussian at every HR pixel, kept where the per-pixel strict test
    |x - s mu_x| < r s W and |y - s mu_y| < r s H holds (density from scipy's
    bivariate normal with covariance L L^T)."""
    oh, ow = _out_size(H, W, s)
    ys, xs = np.meshgrid(np.arange(oh, dtype=np.float64), np.arange(ow, dtype=np.float64),
                         indexing="ij")
    pts = np.stack([xs.ravel() / s, ys.ravel() / s], axis=1)
    img = np.zeros((3, oh * ow))
    masks = []
    for i in range(mean.shape[0]):
        l11, l21, l22 = np.float64(chol[i])
        L = np.array([[l11, 0.0], [l21, l22]])
        m = (np.abs(xs.ravel() - s * float(mean[i, 0])) < r * s * W) & \
            (np.abs(ys.ravel() - s * float(mean[i, 1])) < r * s * H)
        masks.append(m.reshape(oh, ow))
        f = multivariate_normal(mean=np.float64(mean[i]), cov=L @ L.T).pdf(pts)
        img += np.where(m, f, 0.0)[None, :] * (float(opacity[i]) * np.float64(color[i]))[:, None]
    return img.reshape(3, oh, ow), masks


def test_window_rect_against_exact_arithmetic():
    """The FP64 window equals {x : s mu - r s W < x < s mu + r s W} computed
    with 60-digit decimals, away from exact ties."""
    getcontext().prec = 60
    rng = np.random.default_rng(21)
    checked = 0
    for _ in range(400):
        H, W = (int(v) for v in rng.integers(8, 300, 2))
        s = float(rng.uniform(1.0, 12.0))
        r = float(rng.choice([0.01, 0.05, 0.1, 0.4]))
        oh, ow = _out_size(H, W, s)
        mx = float(np.float32(rng.uniform(-5, W + 5)))
        my = float(np.float32(rng.uniform(-5, H + 5)))
        ok, rect = O.window_rect(s, ow, oh, H, W, r, mx, my, 0.7, 0.1, 0.6)

        def exact(mu, ext, n):
            c = Decimal(s) * Decimal(mu)
            h = Decimal(r) * Decimal(s) * ext
            lo, hi = c - h, c + h
            if min(abs(lo - lo.to_integral_value()), abs(hi - hi.to_integral_value())) < \
                    Decimal("1e-9"):
                return None
            return (max(0, int(lo.to_integral_value(rounding="ROUND_FLOOR")) + 1),
                    min(n - 1, int(hi.to_integral_value(rounding="ROUND_CEILING")) - 1))
        ex, ey = exact(mx, W, ow), exact(my, H, oh)
        if ex is None or ey is None:
            continue
        checked += 1
        empty = ex[0] > ex[1] or ey[0] > ey[1]
        assert ok == (not empty)
        if ok:
            assert rect == (ex[0], ex[1], ey[0], ey[1])
    assert checked > 350


def test_window_rect_axes_and_invalid():
    # x pairs with W, y with H: a 20 x 40 LR image at s = 2 (40 x 80 HR),
    # r = 0.1, has half-windows 8 (x) and 4 (y) HR pixels: around (20, 20)
    # the strict test keeps 12 < x < 28 and 16 < y < 24
    ok, rect = O.window_rect(2.0, 80, 40, 20, 40, 0.1, 10.0, 10.0, 1.0, 0.0, 1.0)
    assert ok and rect == (13, 27, 17, 23)
    # around (20.5, 20.5): 12.5 < x < 28.5, 16.5 < y < 24.5
    ok, rect = O.window_rect(2.0, 80, 40, 20, 40, 0.1, 10.25, 10.25, 1.0, 0.0, 1.0)
    assert ok and rect == (13, 28, 17, 24)
    # clipped by the bottom border (HR rows 0..39)
    ok, rect = O.window_rect(2.0, 80, 40, 20, 40, 0.1, 10.0, 19.0, 1.0, 0.0, 1.0)
    assert ok and rect == (13, 27, 35, 39)
    # invalid shape: no support even though the window does not use sigma
    assert not O.window_rect(2.0, 80, 40, 20, 40, 0.1, 10.0, 10.0, 0.0, 0.0, 1.0)[0]
    assert not O.window_rect(2.0, 80, 40, 20, 40, 0.1, 10.0, 10.0, 1.0, 0.0, -1.0)[0]
    assert not O.window_rect(2.0, 80, 40, 20, 40, 0.1, float("nan"), 10.0, 1.0, 0.0, 1.0)[0]


@pytest.mark.parametrize("s,r", [(1.0, 0.1), (2.5, 0.1), (4.0, 0.05), (3.7, 0.25)])
def test_window_forward_and_pairs_match_brute_force(s, r):
    H, W = 12, 10
    wl = synth.tiny(H=H, W=W, s=s, seed=22, extra_frac=0.3, sigma=(0.8, 0.5))
    mean = wl.mean.copy()
    mean[0] = (-1.2, 4.0)   # centre left of the image
    got = O.forward(H, W, s, mean, wl.chol, wl.color, wl.opacity, window=r)
    ref, masks = brute_force_window(H, W, s, r, mean, wl.chol, wl.color, wl.opacity)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert O.support_rects(H, W, s, mean, wl.chol, window=r)[1] == sum(int(m.sum()) for m in masks)
    # tile lists from the per-pixel masks
    tw = th = 8
    oh, ow = got.shape[1:]
    tiles_x = (ow + tw - 1) // tw
    counts, lists = O.tile_lists(H, W, s, mean, wl.chol, tw, th, window=r)
    expect = [[] for _ in counts]
    for i, m in enumerate(masks):
        ys, xs = np.nonzero(m)
        for t in sorted(set((y // th) * tiles_x + x // tw for y, x in zip(ys, xs))):
            expect[t].append(i)
    assert np.array_equal(counts, [len(e) for e in expect])
    assert np.array_equal(lists, [i for e in expect for i in e])


def test_full_window_is_the_untruncated_render():
    """With r = 1 and every centre inside the image, the window holds the
    whole image: Eq. 4 summed over all Gaussians at every pixel, with no
    truncation at all (the all-pairs query the ratio exists to avoid)."""
    H, W, s = 7, 9, 2.7
    wl = synth.tiny(H=H, W=W, s=s, seed=23)
    got = O.forward(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity, window=1.0)
    oh, ow = got.shape[1:]
    ys, xs = np.meshgrid(np.arange(oh) / s, np.arange(ow) / s, indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1)
    ref = np.zeros((3, oh * ow))
    for i in range(wl.n_gauss):
        l11, l21, l22 = np.float64(wl.chol[i])
        L = np.array([[l11, 0.0], [l21, l22]])
        f = multivariate_normal(mean=np.float64(wl.mean[i]), cov=L @ L.T).pdf(pts)
        ref += f[None, :] * (float(wl.opacity[i]) * np.float64(wl.color[i]))[:, None]
    assert np.abs(got - ref.reshape(got.shape)).max() <= 1e-12 * np.abs(ref).max()
    # and it holds more than the 3-sigma box render
    assert (got > O.forward(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity)).any()


def test_window_gradients_match_central_differences():
    H, W, s, r = 6, 7, 2.3, 0.15
    wl = synth.tiny(H=H, W=W, s=s, seed=24)
    oh, ow = _out_size(H, W, s)
    G = np.random.default_rng(24).normal(size=(3, oh, ow))
    m, c, col, op = (np.float64(a).copy() for a in (wl.mean, wl.chol, wl.color, wl.opacity))
    grads = O.backward(H, W, s, m, c, col, op, G, window=r)

    def loss():
        return float((G * O.forward(H, W, s, m, c, col, op, window=r)).sum())

    def rects():
        return O.support_rects(H, W, s, m, c, window=r)[0]
    base = rects()
    checked = skipped = 0
    worst = 0.0
    for arr, grad in zip((m, c, col, op), grads):
        flat, gflat = arr.reshape(-1), grad.reshape(-1)
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            old = flat[j]
            flat[j] = old + h
            lp, rp = loss(), rects()
            flat[j] = old - h
            lm, rm = loss(), rects()
            flat[j] = old
            if not (np.array_equal(rp, base) and np.array_equal(rm, base)):
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            worst = max(worst, abs(fd - gflat[j]) / max(abs(fd), 1e-3))
            checked += 1
    assert skipped <= 0.02 * (checked + skipped)
    assert worst < 1e-6, worst
