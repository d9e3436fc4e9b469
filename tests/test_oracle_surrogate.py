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
