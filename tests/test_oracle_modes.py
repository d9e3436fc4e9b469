"""Pins of the oracle's alternative readings of Eq. 4 and of the truncation:
pixel-centre sampling (HR pixel x samples u = (x + 1/2)/s - 1/2) and the
elliptical support (Mahalanobis distance d < R inside the box).  Each is
checked against an independent route: a brute force with scipy's density
and numpy's inverse covariance, an exact identity between the two sampling
conventions, 60-digit box bounds, the closed-form mass of a truncated
Gaussian, and finite differences."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import synth
from oracle import oracle as O

PC, EL = O.PIXEL_CENTER, O.ELLIPSE


def _out_size(H, W, s):
    return int(math.floor(s * H + 0.5)), int(math.floor(s * W + 0.5))


def brute(H, W, s, mean, chol, color, opacity, mode, R=3.0):
    """Every Gaussian at every HR pixel; membership by the per-pixel box test
    on the sampled LR coordinate and, with the ellipse, d^2 = d^T Sigma^-1 d
    < R^2 from numpy's inverse.  Returns (image, masks, near) where `near`
    marks pixels within 1e-9 of either boundary (left out of exact checks)."""
    oh, ow = _out_size(H, W, s)
    ys, xs = np.meshgrid(np.arange(oh, dtype=np.float64), np.arange(ow, dtype=np.float64),
                         indexing="ij")
    c = 0.5 if mode & PC else 0.0
    u, v = (xs + c) / s - c, (ys + c) / s - c
    pts = np.stack([u.ravel(), v.ravel()], axis=1)
    img = np.zeros((3, oh * ow))
    masks, near = [], np.zeros(oh * ow, bool)
    for i in range(mean.shape[0]):
        l11, l21, l22 = np.float64(chol[i])
        L = np.array([[l11, 0.0], [l21, l22]])
        cov = L @ L.T
        sx, sy = l11, math.hypot(l21, l22)
        mx, my = np.float64(mean[i])
        du, dv = u.ravel() - mx, v.ravel() - my
        m = (np.abs(du) < R * sx) & (np.abs(dv) < R * sy)
        near |= (np.abs(np.abs(du) - R * sx) < 1e-9) | (np.abs(np.abs(dv) - R * sy) < 1e-9)
        if mode & EL:
            d = np.stack([du, dv], axis=1)
            d2 = np.einsum("ij,jk,ik->i", d, np.linalg.inv(cov), d)
            near |= np.abs(d2 - R * R) < 1e-9
            m &= d2 < R * R
        masks.append(m.reshape(oh, ow))
        f = multivariate_normal(mean=[mx, my], cov=cov).pdf(pts)
        img += np.where(m, f, 0.0)[None, :] * (float(opacity[i]) * np.float64(color[i]))[:, None]
    return img.reshape(3, oh, ow), masks, near.reshape(oh, ow)


@pytest.mark.parametrize("mode", [PC, EL, PC | EL])
@pytest.mark.parametrize("s", [1.0, 2.5, 3.7])
def test_modes_match_brute_force(mode, s):
    H, W = 9, 8
    wl = synth.tiny(H=H, W=W, s=s, seed=41, extra_frac=0.3, sigma=(0.7, 0.4))
    got = O.forward(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity, mode=mode)
    ref, masks, near = brute(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity, mode)
    ok = ~near[None]
    assert np.abs(got - ref)[np.broadcast_to(ok, got.shape)].max() <= \
        1e-12 * max(1.0, np.abs(ref).max())
    n_ref = sum(int(m.sum()) for m in masks)
    n_got = O.support_rects(H, W, s, wl.mean, wl.chol, mode=mode)[1]
    assert abs(n_got - n_ref) <= int(near.sum()) * wl.n_gauss
    if not near.any():
        assert n_got == n_ref
    # the ellipse keeps strictly fewer pixels than the box
    if mode & EL:
        assert n_got < O.support_rects(H, W, s, wl.mean, wl.chol, mode=mode & PC)[1]


def test_pixel_centre_is_a_shift_of_the_centre():
    """(x + 1/2)/s - 1/2 - mu = x/s - (mu + 1/2 - 1/(2s)): the pixel-centre
    render of mu is the literal render of mu + 1/2 - 1/(2s) (away from box
    boundary ties, which the two operation sequences may round apart)."""
    H, W, s = 10, 7, 3.3
    wl = synth.tiny(H=H, W=W, s=s, seed=42)
    a = O.forward(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity, mode=PC)
    shifted = np.float64(wl.mean) + 0.5 - 0.5 / s
    b = O.forward(H, W, s, shifted, wl.chol, wl.color, wl.opacity)
    close = np.abs(a - b) <= 1e-12 * np.abs(b).max()
    assert close.mean() > 0.995
    # and s = 1 reduces both conventions to the same sampling
    c1 = O.forward(H, W, 1.0, wl.mean, wl.chol, wl.color, wl.opacity, mode=PC)
    c0 = O.forward(H, W, 1.0, wl.mean, wl.chol, wl.color, wl.opacity)
    assert np.abs(c1 - c0).max() <= 1e-12 * np.abs(c0).max()


def test_pixel_centre_box_against_exact_arithmetic():
    getcontext().prec = 60
    rng = np.random.default_rng(43)
    checked = 0
    for _ in range(300):
        s = float(rng.uniform(1.0, 12.0))
        mx, my = (float(np.float32(v)) for v in rng.uniform(-3, 40, 2))
        l11, l22 = (float(np.float32(v)) for v in np.exp(rng.normal(np.log(0.7), 0.5, 2)))
        l21 = float(np.float32(rng.normal(0, 0.5)))
        ok, r = O.support_rect_m(s, 200, 200, mx, my, l11, l21, l22, 3.0, PC)
        S = Decimal(s)
        sdx = Decimal(l11)
        sdy = (Decimal(l21) ** 2 + Decimal(l22) ** 2).sqrt()

        def exact(mu, sd):
            lo = S * (Decimal(mu) - 3 * sd + Decimal("0.5")) - Decimal("0.5")
            hi = S * (Decimal(mu) + 3 * sd + Decimal("0.5")) - Decimal("0.5")
            if min(abs(lo - lo.to_integral_value()), abs(hi - hi.to_integral_value())) < \
                    Decimal("1e-9"):
                return None
            return (max(0, int(lo.to_integral_value(rounding="ROUND_FLOOR")) + 1),
                    min(199, int(hi.to_integral_value(rounding="ROUND_CEILING")) - 1))
        ex, ey = exact(mx, sdx), exact(my, sdy)
        if ex is None or ey is None:
            continue
        checked += 1
        empty = ex[0] > ex[1] or ey[0] > ey[1]
        assert ok == (not empty)
        if ok:
            assert r == (ex[0], ex[1], ey[0], ey[1])
    assert checked > 250


def test_pixel_d2_is_the_quadratic_form():
    rng = np.random.default_rng(44)
    for _ in range(200):
        s = float(rng.uniform(1, 8))
        mode = int(rng.choice([0, PC]))
        mx, my = rng.uniform(0, 10, 2)
        l11, l22 = np.exp(rng.normal(0, 0.5, 2))
        l21 = rng.normal(0, 0.7)
        x, y = (int(v) for v in rng.integers(0, 80, 2))
        c = 0.5 if mode else 0.0
        d = np.array([(x + c) / s - c - mx, (y + c) / s - c - my])
        L = np.array([[l11, 0], [l21, l22]])
        ref = d @ np.linalg.inv(L @ L.T) @ d
        got = O.pixel_d2(x, y, s, mode, mx, my, l11, l21, l22)
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_elliptical_mass():
    """For an isotropic Gaussian at large s, sum_p I_p / s^2 tends to
    alpha c (1 - exp(-R^2 / 2)) (mass within Mahalanobis radius R), against
    alpha c erf(3 / sqrt 2)^2 for the 3-sigma box."""
    s, sig = 40.0, 0.6
    mu = np.array([[4.1, 3.9]])
    chol = np.array([[sig, 0.0, sig]])
    col, al = np.array([[1.0, 0.5, 0.25]]), np.array([0.8])
    img = O.forward(8, 8, s, mu, chol, col, al, mode=EL)
    mass = img.sum(axis=(1, 2)) / (s * s)
    np.testing.assert_allclose(mass, 0.8 * col[0] * (1 - math.exp(-4.5)), rtol=2e-3)
    box = O.forward(8, 8, s, mu, chol, col, al).sum(axis=(1, 2)) / (s * s)
    np.testing.assert_allclose(box, 0.8 * col[0] * math.erf(3 / math.sqrt(2)) ** 2, rtol=2e-3)


def test_mode_gradients_match_central_differences():
    H, W, s = 6, 6, 2.7
    for mode in (PC, EL, PC | EL):
        wl = synth.tiny(H=H, W=W, s=s, seed=45)
        oh, ow = _out_size(H, W, s)
        G = np.random.default_rng(46).normal(size=(3, oh, ow))
        m, c, col, op = (np.float64(a).copy() for a in (wl.mean, wl.chol, wl.color, wl.opacity))
        grads = O.backward(H, W, s, m, c, col, op, G, mode=mode)

        def loss():
            return float((G * O.forward(H, W, s, m, c, col, op, mode=mode)).sum())

        def support():
            return O.support_rects(H, W, s, m, c, mode=mode)
        base = support()
        checked = skipped = 0
        worst = 0.0
        for arr, grad in zip((m, c, col, op), grads):
            flat, gflat = arr.reshape(-1), grad.reshape(-1)
            for j in range(flat.size):
                h = 1e-6 * max(1.0, abs(flat[j]))
                old = flat[j]
                flat[j] = old + h
                lp, sp = loss(), support()
                flat[j] = old - h
                lm, sm = loss(), support()
                flat[j] = old
                # the support moved (box or ellipse membership): skip
                if not (np.array_equal(sp[0], base[0]) and np.array_equal(sm[0], base[0])
                        and sp[1] == base[1] and sm[1] == base[1]):
                    skipped += 1
                    continue
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(fd - gflat[j]) / max(abs(fd), 1e-3))
                checked += 1
        assert skipped <= 0.05 * (checked + skipped), (mode, skipped)
        assert worst < 1e-6, (mode, worst)


def test_window_pixel_centre_rect():
    # 20 x 40 LR at s = 2 (40 x 80 HR), r = 0.1: half-windows 8 and 4 HR pixels
    # around the pixel-centre HR centre s (mu + 1/2) - 1/2 = (20.5, 20.5)
    ok, rect = O.window_rect(2.0, 80, 40, 20, 40, 0.1, 10.0, 10.0, 1.0, 0.0, 1.0, PC)
    assert ok and rect == (13, 28, 17, 24)
