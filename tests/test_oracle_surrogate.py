"""Pins of the surrogate oracle (labels, BF16 rounding, MLP, loss, Adam)."""
import math

import numpy as np
import pytest
import torch
from scipy.stats import multivariate_normal

import synth
from oracle import oracle as O
from oracle import surrogate as S


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000) * 10 ** rng.uniform(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 65504.0]])
    x = x.astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x), ref)


def test_labels_brute_force():
    """Labels = max Mahalanobis distance over in-box pixels whose single
    contribution alpha max(c) f >= tau, recomputed with scipy's density and a
    linear solve for the distance."""
    H, W, s, tau = 6, 7, 3.3, 2e-3
    wl = synth.tiny(H=H, W=W, s=s, seed=31, sigma=(0.8, 0.5))
    R = O.radius_labels(H, W, s, wl.mean, wl.chol, wl.color, wl.opacity, tau)
    oh, ow = O.output_size(H, W, s)
    rects, _ = O.support_rects(H, W, s, wl.mean, wl.chol)
    for i in range(wl.n_gauss):
        l11, l21, l22 = np.float64(wl.chol[i])
        L = np.array([[l11, 0.0], [l21, l22]])
        mu = np.float64(wl.mean[i])
        x0, x1, y0, y1 = rects[i]
        best = 0.0
        for y in range(y0, y1 + 1):
            for x in range(x0, x1 + 1):
                p = np.array([x / s, y / s])
                f = multivariate_normal(mean=mu, cov=L @ L.T).pdf(p)
                if np.float64(wl.opacity[i]) * np.float64(wl.color[i]).max() * f >= tau:
                    z = np.linalg.solve(L, p - mu)
                    best = max(best, math.sqrt(z @ z))
        assert abs(R[i] - best) < 1e-9, i


def test_labels_approach_closed_form():
    """Dense sampling (large s) of one isotropic Gaussian: the label tends to
    the distance where alpha c K exp(-d^2/2) = tau, K = 1/(2 pi sigma^2)."""
    sig, al, c, tau = 0.9, 0.8, 0.9, 5e-3
    K = 1.0 / (2 * math.pi * sig * sig)
    Rstar = math.sqrt(2 * math.log(al * c * K / tau))
    R = O.radius_labels(12, 12, 40.0, [[6.0, 6.0]], [[sig, 0.0, sig]], [[c, 0.1, 0.2]], [al], tau)
    assert Rstar - 0.05 < R[0] <= Rstar + 1e-12


def _torch_mlp(params, X):
    p = S.unpack(params)
    t = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in p.items()}
    x = torch.tensor(np.asarray(X, np.float64))
    h1 = torch.relu(x @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    out = (h2 @ t["W3"].T)[:, 0] + t["b3"][0]
    return out, t


def test_mlp_exact_mode_matches_torch_autograd():
    """With BF16 rounding switched off, forward and backward equal a float64
    torch MLP and its autograd gradients (an independent derivation)."""
    params = S.init_params(3)
    X = np.random.default_rng(4).normal(size=(257, 8))
    out, cache = S.mlp_forward(params, X, rounding=False)
    tout, t = _torch_mlp(params, X)
    np.testing.assert_allclose(out, tout.detach().numpy(), rtol=1e-12, atol=1e-12)
    dout = np.random.default_rng(5).normal(size=257)
    g = S.mlp_backward(cache, dout, rounding=False)
    (tout * torch.tensor(dout)).sum().backward()
    ref = S.pack({k: v.grad.numpy() for k, v in t.items()})
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-12)


def test_mlp_rounded_mode_stays_within_bf16_error():
    params = S.init_params(7)
    X = np.random.default_rng(8).normal(size=(300, 8))
    a, _ = S.mlp_forward(params, X, rounding=True)
    b, _ = S.mlp_forward(params, X, rounding=False)
    scale = np.abs(b).max()
    assert np.abs(a - b).max() < 0.05 * scale
    assert np.abs(a - b).max() > 0.0  # rounding does happen


def test_pinball_gradient():
    rng = np.random.default_rng(1)
    pred, lab = rng.normal(size=100), rng.normal(size=100)
    for q in (0.5, 0.9):
        loss, g = S.pinball(pred, lab, q)
        h = 1e-7
        for j in range(0, 100, 17):
            pp, pm = pred.copy(), pred.copy()
            pp[j] += h
            pm[j] -= h
            fd = (S.pinball(pp, lab, q)[0] - S.pinball(pm, lab, q)[0]) / (2 * h)
            assert abs(fd - g[j]) < 1e-6
        if q == 0.5:
            assert abs(loss - 0.5 * np.abs(lab - pred).mean()) < 1e-12


def test_adam_matches_torch():
    rng = np.random.default_rng(2)
    p0 = rng.normal(size=50).astype(np.float32)
    tp = torch.tensor(np.float64(p0), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50, np.float32), np.zeros(50, np.float32)
    for t in range(1, 4):
        g = rng.normal(size=50)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = S.adam(p, g, m, v, t, 1e-2)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-6, atol=1e-7)


def test_prune_radius_rules():
    F = np.array([[0.0, 0.0], [2.0, 0.0], [0.5, 0.5]])
    R = S.prune_radius(np.array([1.0, 1.0, 3.5]), 0.2, F, np.array([-1.0, -1.0]),
                       np.array([1.0, 1.0]))
    np.testing.assert_allclose(R, [1.2, 3.0, 3.0])


def test_features_from_constructed_covariance():
    """The features follow from the covariance itself, not from the Cholesky
    factor's entries: build Sigma = R(theta) diag(s1^2, s2^2) R(theta)^T in
    FP64, read sigma_x = sqrt(Sxx), sigma_y = sqrt(Syy), rho = Sxy / (sigma_x
    sigma_y) off it, factor it with numpy's Cholesky and feed the factor to
    the oracle.  Includes strongly anisotropic, rotated Gaussians whose l21 is
    far larger than l22 (where sigma_y and l22 differ most)."""
    rng = np.random.default_rng(12)
    n = 400
    s1 = np.exp(rng.normal(np.log(0.8), 0.7, n))
    s2 = np.exp(rng.normal(np.log(0.8), 0.7, n))
    th = rng.uniform(0.0, np.pi, n)
    s1[:40], s2[:40], th[:40] = 3.0, 0.05, np.pi / 4 + rng.uniform(-0.1, 0.1, 40)
    scale = rng.uniform(1.5, 12.0, n)
    color = rng.uniform(0.0, 1.0, (n, 3))
    alpha = rng.uniform(0.5, 1.0, n)
    chol = np.zeros((n, 3))
    expect = np.zeros((n, 8))
    for i in range(n):
        c, s = math.cos(th[i]), math.sin(th[i])
        Rm = np.array([[c, -s], [s, c]])
        Sig = Rm @ np.diag([s1[i] ** 2, s2[i] ** 2]) @ Rm.T
        L = np.linalg.cholesky(Sig)
        chol[i] = (L[0, 0], L[1, 0], L[1, 1])
        sx, sy = math.sqrt(Sig[0, 0]), math.sqrt(Sig[1, 1])
        expect[i] = (math.log(scale[i]), math.log(sx), math.log(sy), Sig[0, 1] / (sx * sy),
                     alpha[i], *color[i])
    assert (np.abs(chol[:40, 1]) > 5 * chol[:40, 2]).all()
    got = S.features(scale, chol, color, alpha)
    np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-12)


# ---- BF16 rounding points of the MLP, pinned by the BF16 format itself ----
#
# BF16 keeps 8 significant bits: on [1, 2) its spacing is 2^-7, so 1 + 2^-9
# (a quarter of a spacing above 1) rounds to 1, 1 + 2^-8 (a tie) rounds to
# the even neighbour 1, and 1 + 2^-8 + 2^-9 rounds up to 1 + 2^-7.  Each case
# below is a chain network (one live unit per layer) that puts a
# non-representable value at exactly one rounding point.  Where a later
# rounding follows, the next layer's bias adds 2^-8, so that the value there
# is a tie when the earlier rounding happened (result 1) and lies above the
# tie when it did not (result 1 + 2^-7): a missing rounding cannot be hidden
# by the next one.  Expected results are worked out by hand from the spacing.

def _chain(w1=1.0, b1=0.0, w2=1.0, b2=0.0, w3=1.0, b3=0.0):
    d = {"W1": np.zeros((64, 8)), "b1": np.zeros(64), "W2": np.zeros((64, 64)),
         "b2": np.zeros(64), "W3": np.zeros((1, 64)), "b3": np.zeros(1)}
    d["W1"][0, 0], d["b1"][0], d["W2"][0, 0] = w1, b1, w2
    d["b2"][0], d["W3"][0, 0], d["b3"][0] = b2, w3, b3
    return S.pack(d)


def _x(v):
    X = np.zeros((1, 8))
    X[0, 0] = v
    return X


Q = 2.0 ** -9
T = 2.0 ** -8


@pytest.mark.parametrize("point,params,x,rounded,exact", [
    ("input x", _chain(b1=T), 1 + Q, 1.0, 1 + Q + T),
    ("weight W1", _chain(w1=1 + Q, b1=T), 1.0, 1.0, 1 + Q + T),
    ("hidden H1", _chain(b1=Q, b2=T), 1.0, 1.0, 1 + Q + T),
    ("weight W2", _chain(w2=1 + Q, b2=T), 1.0, 1.0, 1 + Q + T),
    ("hidden H2", _chain(b2=Q), 1.0, 1.0, 1 + Q),
    ("weight W3", _chain(w3=1 + Q), 1.0, 1.0, 1 + Q),
    ("output bias (not rounded)", _chain(b3=Q), 1.0, 1 + Q, 1 + Q),
    ("tie above the midpoint", _chain(b1=T + Q), 1.0, 1 + 2 * T, 1 + T + Q),
])
def test_forward_rounding_points(point, params, x, rounded, exact):
    out_r, _ = S.mlp_forward(params, _x(x), rounding=True)
    out_e, _ = S.mlp_forward(params, _x(x), rounding=False)
    assert out_r[0] == rounded, point
    assert out_e[0] == exact, point


def test_backward_rounding_points():
    """d3 (the upstream gradient fed to the matrix cores), dZ2 and dZ1 are
    rounded before they multiply; the bias gradients use the unrounded
    values."""
    P7 = 2.0 ** -7
    # d3: dout = 1 + 2^-9 -> 1 for dW3 (H2 = 1), while db3 sums dout itself
    params = _chain()
    _, cache = S.mlp_forward(params, _x(1.0))
    g = S.unpack(S.mlp_backward(cache, np.array([1 + Q])))
    assert g["W3"][0, 0] == 1.0 and g["b3"][0] == 1 + Q
    # dZ2 = d3b * W3b = (1 + 2^-7)^2 = 1 + 2^-6 + 2^-14 -> 1 + 2^-6 for dW2
    # (H1 = 1); db2 keeps 2^-14; dZ1 = dZ2b * W2b = 1 + 2^-6 -> exact, so
    # dW1 = 1 + 2^-6
    params = _chain(w3=1 + P7)
    _, cache = S.mlp_forward(params, _x(1.0))
    g = S.unpack(S.mlp_backward(cache, np.array([1 + P7])))
    assert g["W2"][0, 0] == 1 + 2 * P7
    assert g["b2"][0] == 1 + 2 * P7 + 2.0 ** -14
    assert g["W1"][0, 0] == 1 + 2 * P7
    # dZ1 = dZ2b * W2b = (1 + 2^-6)(1 + 2^-7) = 1 + 3 * 2^-7 + 2^-13 -> 1 + 3 * 2^-7
    # for dW1 (x = 1); db1 keeps 2^-13
    params = _chain(w2=1 + P7, w3=1 + P7)
    _, cache = S.mlp_forward(params, _x(1.0))
    g = S.unpack(S.mlp_backward(cache, np.array([1 + P7])))
    assert g["W1"][0, 0] == 1 + 3 * P7
    assert g["b1"][0] == 1 + 3 * P7 + 2.0 ** -13
    # without rounding every product keeps its low bits
    g = S.unpack(S.mlp_backward(cache, np.array([1 + P7]), rounding=False))
    assert g["W1"][0, 0] == (1 + P7) ** 3


def test_rounding_is_identity_on_representable_values():
    """Inputs, weights and every intermediate value representable in BF16
    (small integers and powers of two): the rounded MLP equals the exact one
    bit for bit, forward and backward."""
    rng = np.random.default_rng(21)
    d = {"W1": rng.integers(-1, 2, (64, 8)).astype(np.float64),
         "b1": rng.integers(0, 3, 64).astype(np.float64),
         "W2": np.zeros((64, 64)), "b2": rng.integers(0, 3, 64).astype(np.float64),
         "W3": rng.integers(-1, 2, (1, 64)).astype(np.float64), "b3": np.array([0.5])}
    for k in range(64):  # four entries per row keep |Z2| < 256
        d["W2"][k, rng.choice(64, 4, replace=False)] = rng.choice([-1.0, 1.0], 4)
    params = S.pack(d)
    X = rng.integers(-2, 3, (50, 8)).astype(np.float64)
    dout = 2.0 ** rng.integers(-12, -4, 50) * rng.choice([-1.0, 1.0], 50)
    a, ca = S.mlp_forward(params, X, rounding=True)
    b, cb = S.mlp_forward(params, X, rounding=False)
    assert np.array_equal(a, b)
    assert (np.abs(ca[2]).max() > 2) and np.array_equal(ca[2], cb[2])  # H1 nontrivial
    ga = S.mlp_backward(ca, dout, rounding=True)
    gb = S.mlp_backward(cb, dout, rounding=False)
    assert np.array_equal(ga, gb)
    assert np.abs(ga).max() > 0


def test_closed_form_radius_is_where_the_density_reaches_tau():
    """At the closed-form distance R (below the cap), the Gaussian's own
    contribution alpha max(c) f, with f from scipy's bivariate normal density
    at mu + L (R u) for unit vectors u (Mahalanobis distance R), equals tau."""
    rng = np.random.default_rng(3)
    wl = synth.tiny(H=6, W=6, s=2.0, seed=9, sigma=(0.8, 0.5))
    tau = 2e-3
    R = S.closed_form_radius(wl.chol, wl.color, wl.opacity, tau)
    hit = 0
    for i in range(wl.n_gauss):
        if not (0.0 < R[i] < 3.0):
            continue
        l11, l21, l22 = np.float64(wl.chol[i])
        L = np.array([[l11, 0.0], [l21, l22]])
        for th in rng.uniform(0, 2 * np.pi, 3):
            u = np.array([np.cos(th), np.sin(th)])
            p = np.float64(wl.mean[i]) + L @ (R[i] * u)
            f = multivariate_normal(mean=np.float64(wl.mean[i]), cov=L @ L.T).pdf(p)
            val = np.float64(wl.opacity[i]) * np.float64(wl.color[i]).max() * f
            assert abs(val - tau) < 1e-9 * tau
        hit += 1
    assert hit > 10
    assert (S.closed_form_radius(wl.chol, wl.color, wl.opacity, tau, margin=0.3) ==
            np.clip(R + 0.3, 0, 3)).all()
    big = S.closed_form_radius(wl.chol, wl.color, wl.opacity, 1e-30)
    assert (big == 3.0).all()
    bad = np.float64(wl.chol[:2]).copy()
    bad[0, 0] = -1.0
    assert S.closed_form_radius(bad, wl.color[:2], wl.opacity[:2], tau)[0] == 3.0
