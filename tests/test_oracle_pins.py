"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes the oracle's own formulas: each checks it against an
independent route (a library density, a closed form, an invariant of Eq. 4,
exact arithmetic, finite differences, or brute-force enumeration).
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import synth
from oracle import oracle as O


def _out_size(H, W, s):
    return int(math.floor(s * H + 0.5)), int(math.floor(s * W + 0.5))


def brute_force(H, W, s, mean, chol, color, opacity, R=3.0):
    """Every Gaussian at every HR pixel (Algorithm 1's double loop).

    Density from scipy's multivariate normal with covariance L L^T (Eq. 2 is
    the bivariate normal density); membership by the strict per-pixel box test
    s*(mu - R*sigma) < x < s*(mu + R*sigma) evaluated pixel by pixel."""
    oh, ow = _out_size(H, W, s)
    mean, chol = np.asarray(mean, np.float64), np.asarray(chol, np.float64)
    color, opacity = np.asarray(color, np.float64), np.asarray(opacity, np.float64)
    ys, xs = np.meshgrid(np.arange(oh, dtype=np.float64), np.arange(ow, dtype=np.float64),
                         indexing="ij")
    pts = np.stack([xs.ravel() / s, ys.ravel() / s], axis=1)
    img = np.zeros((3, oh * ow))
    masks = []
    for i in range(mean.shape[0]):
        l11, l21, l22 = chol[i]
        L = np.array([[l11, 0.0], [l21, l22]])
        cov = L @ L.T
        sx = l11
        sy = math.sqrt(l21 * l21 + l22 * l22)
        inx = (s * (mean[i, 0] - R * sx) < xs.ravel()) & (xs.ravel() < s * (mean[i, 0] + R * sx))
        iny = (s * (mean[i, 1] - R * sy) < ys.ravel()) & (ys.ravel() < s * (mean[i, 1] + R * sy))
        m = inx & iny
        masks.append(m.reshape(oh, ow))
        f = multivariate_normal(mean=mean[i], cov=cov).pdf(pts)
        img += np.where(m, f, 0.0)[None, :] * (opacity[i] * color[i])[:, None]
    return img.reshape(3, oh, ow), masks


@pytest.mark.parametrize("s", [1.0, 1.5, 3.7, 4.0])
def test_forward_matches_all_pairs_brute_force(s):
    wl = synth.tiny(H=7, W=9, s=s, seed=3)
    got = O.forward(7, 9, s, wl.mean, wl.chol, wl.color, wl.opacity)
    ref, _ = brute_force(7, 9, s, wl.mean, wl.chol, wl.color, wl.opacity)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert (got > 0).sum() > 0.5 * got.size


def test_forward_brute_force_with_extra_and_offimage_gaussians():
    wl = synth.tiny(H=6, W=5, s=2.25, seed=11, extra_frac=0.5, sigma=(0.8, 0.5))
    mean = wl.mean.copy()
    mean[0] = (-2.5, 1.0)      # centre left of the image, support partly inside
    mean[1] = (3.0, 7.4)       # centre below the image
    got = O.forward(6, 5, 2.25, mean, wl.chol, wl.color, wl.opacity)
    ref, _ = brute_force(6, 5, 2.25, mean, wl.chol, wl.color, wl.opacity)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_single_isotropic_gaussian_closed_form():
    s, sig, alpha = 3.0, 0.7, 0.8
    col = np.array([[0.2, 0.5, 1.0]])
    mu = np.array([[4.3, 3.6]])
    chol = np.array([[sig, 0.0, sig]])
    img = O.forward(8, 9, s, mu, chol, col, np.array([alpha]))
    oh, ow = img.shape[1:]
    for y in range(oh):
        for x in range(ow):
            dx, dy = x / s - mu[0, 0], y / s - mu[0, 1]
            inside = (abs(dx) < 3 * sig) and (abs(dy) < 3 * sig)
            val = alpha * math.exp(-(dx * dx + dy * dy) / (2 * sig * sig)) / (2 * math.pi * sig * sig)
            for c in range(3):
                exp_v = col[0, c] * val if inside else 0.0
                assert abs(img[c, y, x] - exp_v) <= 1e-14 + 1e-12 * exp_v


def test_eq2_identities_for_cholesky_form():
    """sx sy sqrt(1-rho^2) = l11 l22 and the Eq. 2 quadratic form equals the
    squared norm of L^-1 (dx, dy): checked through rendered values against the
    determinant-based normalisation of the bivariate normal."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        l11, l22 = rng.uniform(0.3, 2.0, 2)
        l21 = rng.uniform(-2, 2)
        sy = math.sqrt(l21 ** 2 + l22 ** 2)
        rho = l21 / sy
        assert abs(l11 * sy * math.sqrt(1 - rho * rho) - l11 * l22) < 1e-12
        L = np.array([[l11, 0], [l21, l22]])
        d = rng.normal(size=2)
        z = np.linalg.solve(L, d)
        q_eq2 = (d[0] ** 2 / l11 ** 2 - 2 * rho * d[0] * d[1] / (l11 * sy) + d[1] ** 2 / sy ** 2) / (1 - rho * rho)
        assert abs(q_eq2 - z @ z) < 1e-10 * max(1, z @ z)


def test_scale_one_is_eq3():
    """s = 1 gives I_LR(x, y) = sum_i G_i(x, y) on the LR grid (Eq. 3)."""
    wl = synth.tiny(H=6, W=7, s=1.0, seed=8)
    img = O.forward(6, 7, 1.0, wl.mean, wl.chol, wl.color, wl.opacity)
    assert img.shape == (3, 6, 7)
    ref, _ = brute_force(6, 7, 1.0, wl.mean, wl.chol, wl.color, wl.opacity)
    np.testing.assert_allclose(img, ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("s", [2.0, 4.0])
def test_integer_scale_nesting(s):
    """For a power-of-two integer s, I_SR(s j, s k; s) = I_LR(j, k): the
    support test scales exactly, so membership agrees pixel for pixel."""
    wl = synth.tiny(H=6, W=6, s=1.0, seed=21)
    lr = O.forward(6, 6, 1.0, wl.mean, wl.chol, wl.color, wl.opacity)
    hr = O.forward(6, 6, s, wl.mean, wl.chol, wl.color, wl.opacity)
    k = int(s)
    np.testing.assert_allclose(hr[:, ::k, ::k], lr, rtol=1e-13, atol=1e-16)


def test_scale_equivariance():
    """I(.; s, mu, L) = s^2 I(.; 1, s mu, s L): Sigma -> s^2 Sigma.  With
    s = 4 every FP64 product in the support test is exact."""
    s = 4.0
    wl = synth.tiny(H=5, W=6, s=s, seed=2)
    a = O.forward(5, 6, s, wl.mean, wl.chol, wl.color, wl.opacity)
    b = O.forward(20, 24, 1.0, np.float64(wl.mean) * s, np.float64(wl.chol) * s, wl.color,
                  wl.opacity)
    np.testing.assert_allclose(a, s * s * b, rtol=1e-12, atol=1e-16)


def test_mass_of_truncated_gaussian():
    """rho = 0: sum_p I_p / s^2 -> alpha c erf(3/sqrt 2)^2 as s grows (the
    pixel sum is a Riemann sum of the truncated density)."""
    s, sig = 64.0, 1.0
    img = O.forward(12, 12, s, [[6.0, 6.0]], [[sig, 0.0, sig]], [[1.0, 0.5, 0.25]], [0.75])
    mass = img.sum(axis=(1, 2)) / (s * s)
    expect = 0.75 * np.array([1.0, 0.5, 0.25]) * math.erf(3 / math.sqrt(2)) ** 2
    assert abs(math.erf(3 / math.sqrt(2)) ** 2 - 0.994608) < 1e-6
    np.testing.assert_allclose(mass, expect, rtol=2e-3)


def test_permutation_additivity_linearity():
    wl = synth.tiny(H=8, W=7, s=2.7, seed=4)
    args = (8, 7, 2.7)
    base = O.forward(*args, wl.mean, wl.chol, wl.color, wl.opacity)
    perm = np.random.default_rng(0).permutation(wl.n_gauss)
    pimg = O.forward(*args, wl.mean[perm], wl.chol[perm], wl.color[perm], wl.opacity[perm])
    np.testing.assert_allclose(pimg, base, rtol=1e-13, atol=1e-16)
    h = wl.n_gauss // 2
    a = O.forward(*args, wl.mean[:h], wl.chol[:h], wl.color[:h], wl.opacity[:h])
    b = O.forward(*args, wl.mean[h:], wl.chol[h:], wl.color[h:], wl.opacity[h:])
    np.testing.assert_allclose(a + b, base, rtol=1e-13, atol=1e-16)
    two = O.forward(*args, wl.mean, wl.chol, wl.color, np.float64(wl.opacity) * 2)
    np.testing.assert_allclose(two, 2 * base, rtol=1e-13, atol=1e-16)
    col = np.float64(wl.color) * np.array([1.0, 0.0, 3.0])
    lin = O.forward(*args, wl.mean, wl.chol, col, wl.opacity)
    np.testing.assert_allclose(lin, base * np.array([1.0, 0.0, 3.0])[:, None, None],
                               rtol=1e-13, atol=1e-16)


def test_output_size_rounding():
    # 64 x 3.7 = 236.8 -> 237 (the non-integer case of the workloads)
    assert O.output_size(64, 64, 3.7) == (237, 237)
    assert O.output_size(48, 48, 4.0) == (192, 192)
    assert O.output_size(512, 512, 4.0) == (2048, 2048)
    assert O.output_size(256, 256, 12.0) == (3072, 3072)
    assert O.output_size(3, 5, 1.5) == (5, 8)     # 4.5 -> 5 (half up), 7.5 -> 8
    with pytest.raises(ValueError):
        O.output_size(0, 5, 2.0)
    with pytest.raises(ValueError):
        O.output_size(5, 5, float("nan"))


def test_support_rect_against_exact_arithmetic():
    """The FP64 box equals the exact-real set {x : s(mu-3sd) < x < s(mu+3sd)}
    computed with 60-digit decimals, away from exact ties."""
    getcontext().prec = 60
    rng = np.random.default_rng(9)
    n_checked = 0
    for _ in range(400):
        s = float(rng.uniform(1.0, 12.0))
        mx, my = (float(np.float32(v)) for v in rng.uniform(-3, 40, 2))
        l11, l22 = (float(np.float32(v)) for v in np.exp(rng.normal(np.log(0.7), 0.5, 2)))
        l21 = float(np.float32(rng.normal(0, 0.5)))
        ow = oh = 200
        ok, r = O.support_rect(s, ow, oh, mx, my, l11, l21, l22)
        S = Decimal(s)
        sdx = Decimal(l11)
        sdy = (Decimal(l21) ** 2 + Decimal(l22) ** 2).sqrt()

        def exact(mu, sd, n):
            lo = S * (Decimal(mu) - 3 * sd)
            hi = S * (Decimal(mu) + 3 * sd)
            if min(abs(lo - lo.to_integral_value()), abs(hi - hi.to_integral_value())) < Decimal("1e-9"):
                return None
            a = max(0, int(lo.to_integral_value(rounding="ROUND_FLOOR")) + 1)
            b = min(n - 1, int(hi.to_integral_value(rounding="ROUND_CEILING")) - 1)
            return a, b
        ex, ey = exact(mx, sdx, ow), exact(my, sdy, oh)
        if ex is None or ey is None:
            continue
        n_checked += 1
        empty = ex[0] > ex[1] or ey[0] > ey[1]
        assert ok == (not empty)
        if ok:
            assert r == (ex[0], ex[1], ey[0], ey[1])
    assert n_checked > 350


def test_support_rect_invalid_inputs():
    assert not O.support_rect(2.0, 10, 10, 1.0, 1.0, 0.0, 0.0, 1.0)[0]
    assert not O.support_rect(2.0, 10, 10, 1.0, 1.0, 1.0, 0.0, -1.0)[0]
    assert not O.support_rect(2.0, 10, 10, float("nan"), 1.0, 1.0, 0.0, 1.0)[0]
    assert not O.support_rect(2.0, 10, 10, 1.0, float("inf"), 1.0, 0.0, 1.0)[0]
    assert not O.support_rect(2.0, 10, 10, 100.0, 1.0, 1.0, 0.0, 1.0)[0]
    # exact tie: s(mu - 3 sd) = 2 is excluded, next integer 3 is the first
    ok, r = O.support_rect(1.0, 20, 20, 5.0, 5.0, 1.0, 0.0, 1.0)
    assert ok and r == (3, 7, 3, 7)


@pytest.mark.parametrize("tw,th", [(4, 4), (8, 4), (3, 5)])
def test_tile_lists_match_enumeration(tw, th):
    """A Gaussian is in tile t iff some in-support pixel lies in t; lists in
    ascending Gaussian index (enumerated from the per-pixel brute-force masks)."""
    H, W, s = 6, 7, 2.6
    wl = synth.tiny(H=H, W=W, s=s, seed=6, extra_frac=0.3)
    counts, lists = O.tile_lists(H, W, s, wl.mean, wl.chol, tw, th)
    _, masks = brute_force(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity)
    oh, ow = _out_size(H, W, s)
    tx_n, ty_n = -(-ow // tw), -(-oh // th)
    expect = []
    for ty in range(ty_n):
        for tx in range(tx_n):
            members = [i for i, m in enumerate(masks)
                       if m[ty * th:(ty + 1) * th, tx * tw:(tx + 1) * tw].any()]
            expect.append(members)
    assert counts.tolist() == [len(e) for e in expect]
    assert lists.tolist() == [i for e in expect for i in e]


def test_tile_lists_batch_layout():
    wl = synth.tiny(H=4, W=5, s=2.0, seed=1, n_images=3)
    ranges, lists = O.tile_lists_batch(wl, 4, 4)
    per = []
    for k, im in enumerate(wl.images):
        sl = wl.image_slice(k)
        c, l = O.tile_lists(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl], 4, 4)
        per.append((c, l + im.g_begin))
    assert ranges.shape[0] == sum(len(c) for c, _ in per)
    assert np.array_equal(lists, np.concatenate([l for _, l in per]))
    for t in range(ranges.shape[0]):
        b, e = ranges[t]
        assert e >= b


def _fd_case(seed=12):
    H, W, s = 6, 6, 2.3
    wl = synth.tiny(H=H, W=W, s=s, seed=seed)
    oh, ow = _out_size(H, W, s)
    G = np.random.default_rng(seed).normal(size=(3, oh, ow))
    return H, W, s, wl, G


def test_gradients_match_central_differences():
    """Analytic gradients of L = sum(G * I) vs FP64 central differences
    (h = 1e-6 max(1, |theta|)); parameters whose support box moves under
    +-h are skipped and counted."""
    H, W, s, wl, G = _fd_case()
    m, c, col, op = (np.float64(a).copy() for a in (wl.mean, wl.chol, wl.color, wl.opacity))
    gm, gc, gcol, gop = O.backward(H, W, s, m, c, col, op, G)

    def loss(m_, c_, col_, op_):
        return float((G * O.forward(H, W, s, m_, c_, col_, op_)).sum())

    def rects(m_, c_):
        return O.support_rects(H, W, s, m_, c_)[0]

    base_rects = rects(m, c)
    checked = skipped = 0
    worst = 0.0
    for arr, grad in ((m, gm), (c, gc), (col, gcol), (op, gop)):
        flat, gflat = arr.reshape(-1), grad.reshape(-1)
        for j in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[j]))
            old = flat[j]
            flat[j] = old + h
            lp, rp = loss(m, c, col, op), rects(m, c)
            flat[j] = old - h
            lm, rm = loss(m, c, col, op), rects(m, c)
            flat[j] = old
            if not (np.array_equal(rp, base_rects) and np.array_equal(rm, base_rects)):
                skipped += 1
                continue
            fd = (lp - lm) / (2 * h)
            err = abs(fd - gflat[j]) / max(abs(fd), 1e-3)
            worst = max(worst, err)
            checked += 1
    assert skipped <= 0.01 * (checked + skipped)
    assert worst < 1e-6, worst


def test_gradient_zero_for_invalid_and_offimage():
    H, W, s, wl, G = _fd_case(seed=13)
    m = np.float64(wl.mean).copy()
    c = np.float64(wl.chol).copy()
    m[0] = (500.0, 500.0)          # support entirely off the image
    c[1, 0] = -1.0                 # invalid l11
    gm, gc, gcol, gop = O.backward(H, W, s, m, c, wl.color, wl.opacity, G)
    for i in (0, 1):
        assert not gm[i].any() and not gc[i].any() and not gcol[i].any() and gop[i] == 0


def test_l1_loss_grad_and_psnr():
    a = [np.array([[0.5, 0.2], [0.1, 0.1]])]
    t = [np.array([[0.0, 0.4], [0.1, 0.3]])]
    loss, g = O.l1_loss_and_grad(a, t)
    assert abs(loss - (0.5 + 0.2 + 0.0 + 0.2) / 4) < 1e-15
    np.testing.assert_array_equal(g[0], np.array([[1, -1], [0, -1]]) / 4)
    x = np.full((3, 4, 4), 0.3)
    assert abs(O.psnr([x + 1e-3], [x]) - 60.0) < 1e-9


def test_pixel_values_equal_full_render():
    wl = synth.tiny(H=9, W=8, s=3.3, seed=17, extra_frac=0.25)
    img = O.forward(9, 8, 3.3, wl.mean, wl.chol, wl.color, wl.opacity)
    rng = np.random.default_rng(1)
    ys = rng.integers(0, img.shape[1], 200)
    xs = rng.integers(0, img.shape[2], 200)
    vals = O.pixel_values(9, 8, 3.3, wl.mean, wl.chol, wl.color, wl.opacity, xs, ys)
    np.testing.assert_allclose(vals, img[:, ys, xs], rtol=1e-13, atol=1e-300)


def test_radius_support_shrinks_box():
    """A per-Gaussian radius R replaces 3 in the box half-width: R = 3 equals
    the default, a smaller R gives a subset of the pixels with identical
    values there (brute force with R)."""
    wl = synth.tiny(H=6, W=7, s=2.9, seed=23)
    n = wl.n_gauss
    a = O.forward(6, 7, 2.9, wl.mean, wl.chol, wl.color, wl.opacity)
    b = O.forward(6, 7, 2.9, wl.mean, wl.chol, wl.color, wl.opacity, radius=np.full(n, 3.0))
    np.testing.assert_array_equal(a, b)
    R = np.random.default_rng(2).uniform(0.5, 3.0, n)
    c = O.forward(6, 7, 2.9, wl.mean, wl.chol, wl.color, wl.opacity, radius=R)
    ref = np.zeros_like(c)
    for i in range(n):
        part, _ = brute_force(6, 7, 2.9, wl.mean[i:i + 1], wl.chol[i:i + 1], wl.color[i:i + 1],
                              wl.opacity[i:i + 1], R=R[i])
        ref += part
    np.testing.assert_allclose(c, ref, rtol=1e-12, atol=1e-300)
    assert (c <= a + 1e-15).all()


@pytest.mark.parametrize("s", [1.0, 2.25, 3.7])
def test_support_pair_count_equals_brute_force_masks(s):
    """The in-support pair count (the work figure of the roofline and the
    n_support the GPU reports) equals the number of (pixel, Gaussian) pairs
    that pass the per-pixel strict box test, counted over brute-force masks,
    with Gaussians partly and wholly off the image and a per-Gaussian radius."""
    H, W = 6, 7
    wl = synth.tiny(H=H, W=W, s=s, seed=41, extra_frac=0.4, sigma=(0.8, 0.5))
    mean = np.float64(wl.mean).copy()
    chol = np.float64(wl.chol).copy()
    chol[:2] = (1.0, 0.3, 0.9)
    mean[0] = (-2.0, 2.0)      # box clipped at the left edge
    mean[1] = (3.0, H + 1.0)   # box clipped at the bottom
    mean[2] = (500.0, 3.0)     # no pixel at all
    _, masks = brute_force(H, W, s, mean, chol, wl.color, wl.opacity)
    rects, total = O.support_rects(H, W, s, mean, chol)
    assert total == sum(int(m.sum()) for m in masks)
    assert masks[2].sum() == 0 and masks[0].sum() > 0 and masks[1].sum() > 0
    for i, m in enumerate(masks):
        x0, x1, y0, y1 = rects[i]
        area = max(0, x1 - x0 + 1) * max(0, y1 - y0 + 1)
        assert area == int(m.sum()), i
    R = np.random.default_rng(3).uniform(0.4, 3.0, wl.n_gauss)
    _, total_r = O.support_rects(H, W, s, mean, chol, R)
    count_r = 0
    for i in range(wl.n_gauss):
        _, mk = brute_force(H, W, s, mean[i:i + 1], chol[i:i + 1], wl.color[i:i + 1],
                            wl.opacity[i:i + 1], R=R[i])
        count_r += int(mk[0].sum())
    assert total_r == count_r
    assert O.support_pairs_batch(wl) == O.support_rects(H, W, s, wl.mean, wl.chol)[1]


def test_multithreaded_oracle_is_bitwise_serial():
    """The OpenMP variants (row bands forward, Gaussians backward) give the
    single-threaded oracle's values bit for bit."""
    wl = synth.tiny(H=40, W=23, s=3.3, seed=5, extra_frac=0.3, sigma=(0.8, 0.5))
    a = O.forward(40, 23, 3.3, wl.mean, wl.chol, wl.color, wl.opacity)
    b = O.forward(40, 23, 3.3, wl.mean, wl.chol, wl.color, wl.opacity, threads=4)
    assert np.array_equal(a, b)
    G = np.random.default_rng(1).normal(size=a.shape)
    ga = O.backward(40, 23, 3.3, wl.mean, wl.chol, wl.color, wl.opacity, G)
    gb = O.backward(40, 23, 3.3, wl.mean, wl.chol, wl.color, wl.opacity, G, threads=4)
    for x, y in zip(ga, gb):
        assert np.array_equal(x, y)


def test_box_cut_by_border_brute_force():
    """The border cuts a support box iff some integer x (or y) passing the
    strict window test s(mu - 3 sd) < x < s(mu + 3 sd) lies outside the
    image; enumerated integer by integer over a wide range."""
    H, W, s = 6, 7, 2.6
    wl = synth.tiny(H=H, W=W, s=s, seed=13, extra_frac=0.5, sigma=(0.8, 0.5))
    oh, ow = _out_size(H, W, s)
    cut = O.box_cut(H, W, s, wl.mean, wl.chol)
    ints = np.arange(-200, 400)
    for i in range(wl.n_gauss):
        l11, l21, l22 = np.float64(wl.chol[i])
        sx, sy = l11, math.sqrt(l21 * l21 + l22 * l22)
        mx, my = np.float64(wl.mean[i])
        xs = ints[(s * (mx - 3 * sx) < ints) & (ints < s * (mx + 3 * sx))]
        ys = ints[(s * (my - 3 * sy) < ints) & (ints < s * (my + 3 * sy))]
        out = (xs < 0).any() or (xs > ow - 1).any() or (ys < 0).any() or (ys > oh - 1).any()
        assert cut[i] == (1 if out else 0), i
    assert 0 < (cut == 1).sum() < wl.n_gauss
