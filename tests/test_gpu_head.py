"""The Gaussian primary head and the Y-channel PSNR kernels against the FP64
oracle (oracle/head.py), element by element.

Head tolerances come from the kernels' FP32 arithmetic: every output is a
short chain of correctly rounded operations and library exp/expm1 calls
(a few ulps each), so each value lies within 32 u (u = 2^-24) of the sum of
the magnitudes of the terms it is formed from (the oracle's own FP64 error is
far below that for raw inputs within +-8); the reference positions and
offsets add once (u |p| + u |mu|)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import head as Hd
from oracle import oracle as O
from tests._gpu import plan_for, say, to_dev

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _raw(n, seed, spread=3.0):
    rng = np.random.default_rng(seed)
    c = lambda a: np.clip(a, -8, 8).astype(np.float32)
    return (c(rng.normal(0, spread, n)), c(rng.normal(0, spread, (n, 3))),
            c(rng.normal(0, spread, (n, 2))), c(rng.normal(0, spread, n)),
            rng.normal(0, 0.6, (n, 2)).astype(np.float32))


def _refpos(images, n):
    P = np.full((n, 2), np.nan)
    for h, w, gb, gc, g in images:
        P[gb:gb + gc] = Hd.reference_positions(h, w, g)
    return P


def _cuda(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _layout(sizes, grid, gap=0):
    out, g = [], 0
    for h, w in sizes:
        n = grid * grid * h * w
        out.append((h, w, g, n))
        g += n + gap
    return out, g


@pytest.mark.parametrize("grid,sizes,gap", [(4, [(5, 7), (3, 4), (12, 9)], 0),
                                            (1, [(16, 16)], 0),
                                            (3, [(2, 5), (7, 3)], 5),
                                            (2, [(1, 1)] * 40, 0)])
def test_head_forward_parity(grid, sizes, gap):
    from paper_2501_06838_amd.head import gaussian_head
    images, n = _layout(sizes, grid, gap)
    say("head forward", grid, sizes, "gap", gap)
    raw = _raw(n, grid * 100 + len(sizes))
    tr = _cuda(*raw)
    mean, chol, color, opacity = gaussian_head(images, grid, *tr)
    torch.cuda.synchronize()
    P = _refpos([im + (grid,) for im in images], n)
    rm, rc, rcol, rop = Hd.head_forward(*[np.float64(a) for a in raw], P)
    inside = ~np.isnan(P[:, 0])
    got = [x.cpu().numpy().astype(np.float64)[inside] for x in (mean, chol, color, opacity)]
    rm, rc, rcol, rop = rm[inside], rc[inside], rcol[inside], rop[inside]
    assert (np.abs(got[3] - rop) <= 32 * U * rop).all()
    assert (np.abs(got[2] - rcol) <= 32 * U * rcol).all()
    assert (np.abs(got[1] - rc) <= 32 * U * np.abs(rc)).all()
    env_mean = np.abs(P[inside]) + np.abs(rm)
    assert (np.abs(got[0] - rm) <= 2 * U * env_mean).all()


def test_head_backward_parity():
    from paper_2501_06838_amd import _native as N
    from paper_2501_06838_amd.raster import _ptr, _stream
    n = 50_000
    raw = _raw(n, 7)
    rng = np.random.default_rng(8)
    G = [rng.normal(size=s).astype(np.float32) for s in [(n, 2), (n, 3), (n, 3), (n,)]]
    say("head backward", n)
    ins = _cuda(*raw[:4], *G)
    outs = [torch.full(s, float("nan"), device="cuda") for s in
            [(n,), (n, 3), (n, 2), (n,), (n, 2)]]
    N.check(N.lib().gs_gaussian_head_backward(n, *[_ptr(t) for t in ins],
                                              *[_ptr(t) for t in outs], _stream()), "bwd")
    torch.cuda.synchronize()
    got = [t.cpu().numpy().astype(np.float64) for t in outs]
    r = [np.float64(a) for a in raw]
    ref = Hd.head_backward(r[0], r[1], r[2], r[3], *[np.float64(g) for g in G])
    # magnitude envelopes of the terms each output is formed from
    sig = lambda x: 1 / (1 + np.exp(-x))
    rho = np.tanh(r[3])
    root = np.sqrt(1 - rho * rho)
    sy = sig(r[2][:, 1])
    g21, g22 = np.float64(G[1][:, 1]), np.float64(G[1][:, 2])
    env = [np.abs(ref[0]), np.abs(ref[1]), np.abs(ref[2]).copy(),
           (np.abs(g21) * root + np.abs(g22) * np.abs(rho)) * sy * root, None]
    env[2][:, 1] = (np.abs(g21 * rho) + np.abs(g22) * root) * sig(r[2][:, 1]) * sig(-r[2][:, 1])
    for k, name in enumerate(("opacity", "color", "sigma", "rho")):
        bad = np.abs(got[k] - ref[k]) > 32 * U * env[k]
        assert not bad.any(), f"{name}: {bad.sum()} outside"
    assert np.array_equal(got[4], np.float64(G[0]))


def test_head_autograd_into_the_rasterizer():
    """Head -> rasterizer forward -> L1 step through autograd: the image
    against the two oracles chained, and the raw-output gradients against
    the oracle's chain (rasterizer backward then head backward)."""
    import paper_2501_06838_amd as G
    from paper_2501_06838_amd.head import gaussian_head
    grid, sizes, s = 2, [(9, 11), (6, 6)], 3.3
    images, n = _layout(sizes, grid)
    raw = list(_raw(n, 9, spread=1.0))
    raw[2] = np.clip(raw[2] + 0.5, -8, 8).astype(np.float32)  # sigma around 0.6 LR px
    say("head into rasterizer", n)
    tr = [t.requires_grad_(True) for t in _cuda(*raw)]
    mean, chol, color, opacity = gaussian_head(images, grid, *tr)
    plan = G.RasterPlan([(h, w, s, gb, gc) for h, w, gb, gc in images], n, tile=16)
    out = G.rasterize(mean, chol, color, opacity, plan)
    rng = np.random.default_rng(10)
    targets = [rng.uniform(0, 1, (3,) + sz).astype(np.float32) for sz in plan.sizes]
    target = plan.pack([torch.from_numpy(t).cuda() for t in targets])
    loss, grad = G.l1_loss_grad(out.detach(), target)
    out.backward(grad)
    torch.cuda.synchronize()
    # oracle chain on the kernel's own FP32 head outputs for the render
    P = _refpos([im + (grid,) for im in images], n)
    om, oc, ocol, oop = (x.detach().cpu().numpy() for x in (mean, chol, color, opacity))
    for k, (h, w, gb, gc) in enumerate(images):
        sl = slice(gb, gb + gc)
        ref = O.forward(h, w, s, om[sl], oc[sl], ocol[sl], oop[sl])
        got = plan.split(out.detach())[k].cpu().numpy()
        err = np.abs(got - ref)
        assert (err <= 1e-5 * np.abs(ref) + 1e-30).all()
    Gs = [x.cpu().double().numpy() for x in plan.split(grad)]
    gm = np.zeros((n, 2)); gc_ = np.zeros((n, 3)); gcol = np.zeros((n, 3)); gop = np.zeros(n)
    for k, (h, w, gb, gc) in enumerate(images):
        sl = slice(gb, gb + gc)
        a, b, c, d = O.backward(h, w, s, om[sl], oc[sl], ocol[sl], oop[sl], Gs[k])
        gm[sl], gc_[sl], gcol[sl], gop[sl] = a, b, c, d
    ref = Hd.head_backward(*[np.float64(a) for a in raw[:4]], gm, gc_, gcol, gop)
    for name, t, r in zip(("opacity", "color", "sigma", "rho", "offset"), tr, ref):
        g = t.grad.cpu().double().numpy()
        scale = np.abs(r).max()
        assert np.abs(g - r).max() <= 1e-3 * scale, name


@pytest.mark.parametrize("crop", [0, 3])
def test_psnr_y_parity(crop):
    from paper_2501_06838_amd.head import psnr_y
    wl = synth.config3(n_images=40)  # two chunks of the by-value image table
    plan = plan_for(wl, 16)
    rng = np.random.default_rng(11)
    ref = [rng.uniform(0, 1, (3,) + sz).astype(np.float32) for sz in plan.sizes]
    noise = [rng.normal(0, 0.01 * (k + 1), r.shape).astype(np.float32) for k, r in enumerate(ref)]
    test = [r + e for r, e in zip(ref, noise)]
    test[5] = ref[5].copy()  # identical image: +inf
    say("psnr y", len(ref), "crop", crop)
    p, sse = psnr_y(plan, plan.pack([torch.from_numpy(t).cuda() for t in test]),
                    plan.pack([torch.from_numpy(r).cuda() for r in ref]), crop=crop)
    p, sse = p.cpu().numpy(), sse.cpu().numpy()
    for k in range(len(ref)):
        rp, rsse, cnt = Hd.psnr_y(test[k], ref[k], crop=crop)
        if k == 5:
            assert p[k] == math.inf and sse[k] == 0.0
            continue
        assert abs(sse[k] - rsse) <= 1e-12 * rsse
        assert abs(p[k] - rp) <= 1e-9


def test_psnr_y_crop_leaves_nothing():
    from paper_2501_06838_amd.head import psnr_y
    wl = synth.tiny(H=3, W=4, s=2.0, n_images=1)
    plan = plan_for(wl, 16)
    a = torch.rand(plan.out_numel, device="cuda")
    p, sse = psnr_y(plan, a, a * 0.5, crop=3)
    assert math.isnan(p.item()) and sse.item() == 0.0
