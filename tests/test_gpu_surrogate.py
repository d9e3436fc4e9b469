"""GPU parity of the learned-radius kernels against the surrogate oracle.

The MLP's operands are rounded to BF16 on both sides at the same points, but
each side forms the value it rounds in its own precision (FP32 accumulation
on the matrix cores, FP64 in the oracle).  Every element is therefore held
to a bound carried through the network from the oracle's own values
(tests/_mlp_bound.py): the FP32 accumulation error of each sum, plus a BF16
spacing only where a rounding boundary or a ReLU's zero lies within the
propagated error of the value being rounded.  Elsewhere (almost everywhere)
the bound is the FP32 accumulation error alone.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from oracle import surrogate as S
from tests import _mlp_bound as B
from tests._gpu import plan_for, render, say, to_dev

pytestmark = pytest.mark.gpu


def _params(seed):
    p = S.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 100)
    d = S.unpack(p)
    d["b1"] = rng.normal(0, 0.3, 64)
    d["b2"] = rng.normal(0, 0.3, 64)
    d["b3"] = rng.normal(0, 0.3, 1)
    return S.pack(d).astype(np.float32)


NAMES = (("W1", slice(0, 512)), ("b1", slice(512, 576)), ("W2", slice(576, 4672)),
         ("b2", slice(4672, 4736)), ("W3", slice(4736, 4800)), ("b3", slice(4800, 4801)))


def _check_bound(got, ref, err, name, tight_share=None):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    bad = np.abs(got - ref) > err
    assert not bad.any(), (f"{name}: {bad.sum()} of {bad.size} elements outside the bound; "
                           f"worst excess {(np.abs(got - ref) - err).max():.3e}")
    if tight_share is not None:
        scale = max(np.abs(ref).max(), 1e-30)
        assert (err <= 1e-4 * scale).mean() >= tight_share, name


@pytest.mark.parametrize("n", [1, 37, 1000, 20000])
def test_mlp_forward_parity(n):
    """Every prediction within its bound; most bounds under 1e-4 of the
    largest prediction (the FP32 accumulation error alone)."""
    from paper_2501_06838_amd.surrogate import RadiusMLP
    params = _params(1)
    X = np.random.default_rng(2 + n).normal(size=(n, 8)).astype(np.float32)
    say("mlp forward", n)
    net = RadiusMLP(params)
    got = net.predict(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    ref, err, _ = B.forward_bound(params, X)
    _check_bound(got, ref, err, "prediction", tight_share=0.5 if n >= 37 else None)


@pytest.mark.parametrize("n", [1, 37, 1000, 20000])
def test_mlp_gradient_parity(n):
    """Every parameter's gradient for a given upstream gradient within its
    bound (the batch sums accumulate in FP32 in the kernel's order)."""
    from paper_2501_06838_amd.surrogate import RadiusMLP
    params = _params(3)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(n, 8)).astype(np.float32)
    dout = (rng.normal(size=n) / n).astype(np.float32)
    say("mlp grad", n)
    net = RadiusMLP(params)
    g = net.gradient(torch.from_numpy(X).cuda(), dout=torch.from_numpy(dout).cuda())
    g = g.cpu().numpy().astype(np.float64)
    _, _, st = B.forward_bound(params, X)
    ref, err = B.backward_bound(st, np.asarray(dout, np.float64), np.zeros(n))
    for name, sl in NAMES:
        _check_bound(g[sl], ref[sl], err[sl], name)


def test_mlp_pinball_gradient():
    """The pinball loss's value and gradient within their bounds (rows whose
    label lies within the prediction's bound may take either branch)."""
    from paper_2501_06838_amd.surrogate import RadiusMLP
    params = _params(5)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(4096, 8)).astype(np.float32)
    lab = rng.uniform(0, 3, 4096).astype(np.float32)
    say("mlp pinball")
    net = RadiusMLP(params)
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    g = net.gradient(torch.from_numpy(X).cuda(), labels=torch.from_numpy(lab).cuda(),
                     quantile=0.9, loss=loss)
    g = g.cpu().numpy().astype(np.float64)
    pred, epred, st = B.forward_bound(params, X)
    ref_loss, _ = S.pinball(pred, lab, 0.9)
    # |d loss / d pred| <= max(q, 1 - q) / n per row, plus FP32 rounding of
    # the per-row terms and their sum
    e_loss = 0.9 * epred.sum() / lab.size + 1e-6 * abs(ref_loss)
    assert abs(loss.item() - ref_loss) <= e_loss
    d, ed = B.pinball_upstream(st, lab, 0.9)
    ref, err = B.backward_bound(st, d, ed)
    for name, sl in NAMES:
        _check_bound(g[sl], ref[sl], err[sl], name)


def _adam_bounds(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Per-element radii of the kernel's FP32 Adam step (same FP32 inputs)
    around the oracle's FP64 step.  The kernel holds b1, b2 and lr as FP32
    numbers (their distance to the FP64 constants counts in full), rounds each
    product and sum once (u = 2^-24), and takes powf and sqrtf within a few
    ulps (4u is allowed for each)."""
    u = 2.0 ** -24
    p, m, v, g = (np.asarray(a, np.float64) for a in (p, m, v, g))
    b1f, b2f, lrf = float(np.float32(b1)), float(np.float32(b2)), float(np.float32(lr))
    m1 = b1 * m + (1 - b1) * g
    v1 = b2 * v + (1 - b2) * g * g
    e_m = abs(b1f - b1) * (np.abs(m) + np.abs(g)) + 2 * u * (np.abs(b1 * m) + np.abs((1 - b1) * g))
    e_v = abs(b2f - b2) * (v + g * g) + 3 * u * (b2 * v + (1 - b2) * g * g)
    d1, d2 = 1 - b1 ** t, 1 - b2 ** t
    rel_d1 = (4 * u * b1 ** t + t * abs(b1f - b1)) / d1 + u
    rel_d2 = (4 * u * b2 ** t + t * abs(b2f - b2)) / d2 + u
    mh, vh = m1 / d1, v1 / d2
    e_mh = e_m / d1 * (1 + rel_d1) + np.abs(mh) * (rel_d1 + u)
    e_vh = e_v / d2 * (1 + rel_d2) + vh * (rel_d2 + u)
    sq = np.sqrt(vh)
    e_sq = e_vh / (2 * np.maximum(sq, 1e-300)) + 4 * u * sq
    den = sq + eps
    e_den = e_sq + u * den
    upd = lr * mh / den
    e_upd = abs(lrf - lr) * np.abs(mh) / den + lr * (
        e_mh / den + np.abs(mh) * e_den / (den * (den - e_den))) + 3 * u * np.abs(upd)
    p1 = p - upd
    e_p = e_upd + u * np.abs(p1)
    return e_p, e_m, e_v


def test_mlp_adam_step():
    """Adam steps of the kernel against the oracle's, each from the same FP32
    weights, moments and gradient, within the radii of the FP32 arithmetic."""
    from paper_2501_06838_amd.surrogate import RadiusMLP
    import ctypes
    from paper_2501_06838_amd import _native as N
    from paper_2501_06838_amd.raster import _ptr, _stream
    from paper_2501_06838_amd.surrogate import _bind
    rng = np.random.default_rng(7)
    params = _params(5)
    g = (rng.normal(size=4801) * 1e-2).astype(np.float32)
    m0 = (rng.normal(size=4801) * 1e-3).astype(np.float32)
    v0 = (rng.uniform(0, 1e-4, 4801)).astype(np.float32)
    say("adam")
    net = RadiusMLP(params)
    gd = torch.from_numpy(g).cuda()
    L = _bind()
    for t, lr in ((1, 1e-3), (7, 3e-3), (1000, 1e-2)):
        net.params.copy_(torch.from_numpy(np.asarray(params, np.float32)))
        net.m.copy_(torch.from_numpy(m0))
        net.v.copy_(torch.from_numpy(v0))
        N.check(L.gs_mlp_adam(_ptr(net.params), _ptr(net.m), _ptr(net.v), _ptr(gd), t,
                              ctypes.c_float(lr), _stream()), "adam")
        e_p, e_m, e_v = _adam_bounds(params, m0, v0, g, t, lr)
        p1, m1, v1 = S.adam(params, g, m0, v0, t, lr, exact=True)
        for name, got, ref, err in (("params", net.params, p1, e_p), ("m", net.m, m1, e_m),
                                    ("v", net.v, v1, e_v)):
            got = got.cpu().numpy().astype(np.float64)
            bad = np.abs(got - ref) > err
            assert not bad.any(), f"t={t} {name}: {bad.sum()} outside the bound"
            # the bound is tight: the FP32 step moves the weights by far more
            if name == "params":
                assert np.median(err / np.maximum(np.abs(p1 - params), 1e-30)) < 1e-3
        # the next step starts from the oracle's FP32 state
        params, m0, v0 = S.adam(params, g, m0, v0, t, lr)


def test_features_parity():
    from paper_2501_06838_amd.surrogate import features, make_norm
    wl = synth.config3(n_images=40)   # two chunks of the by-value image table
    plan = plan_for(wl, 16)
    m, c, col, op = to_dev(wl)
    scale = np.concatenate([np.full(im.g_count, im.scale) for im in wl.images])
    F = S.features(scale, wl.chol, wl.color, wl.opacity)
    mu, sd = F.mean(0), F.std(0)
    say("features")
    got = features(plan, c, col, op, make_norm(mu, sd)).cpu().numpy()
    ref = (F - mu) / sd
    assert np.abs(got - ref).max() < 1e-5 * max(1.0, np.abs(ref).max())


def test_radius_labels_bracket_oracle():
    """GPU labels decide 'contribution >= tau' in FP32: each must lie between
    the oracle's labels at tau (1 + 1e-4) and tau (1 - 1e-4)."""
    from paper_2501_06838_amd.surrogate import radius_labels
    wl = synth.tiny(H=24, W=20, s=5.3, seed=8, sigma=(0.8, 0.5), extra_frac=0.25)
    tau = 2e-3
    say("radius stats")
    plan, ws, _ = render(wl, 16)
    got = radius_labels(plan, ws, tau).cpu().numpy().astype(np.float64)
    lo = O.radius_labels_batch(wl, tau * (1 + 1e-4))
    hi = O.radius_labels_batch(wl, tau * (1 - 1e-4))
    assert (got >= lo * (1 - 1e-5) - 1e-6).all() and (got <= hi * (1 + 1e-5) + 1e-6).all()
    assert (got > 0).mean() > 0.5
    # interior only: -1 exactly where the oracle finds the box cut by the border
    gi = radius_labels(plan, ws, tau, interior_only=True).cpu().numpy().astype(np.float64)
    ref_i = O.interior_labels_batch(wl, tau)
    assert np.array_equal(gi < 0, ref_i < 0)
    assert 0 < (gi < 0).sum() < gi.size
    keep = gi >= 0
    assert np.array_equal(gi[keep], got[keep])


def test_closed_form_radius_parity():
    """The control's closed-form radius (FP64 in the kernel) against the
    oracle's, with a margin and invalid entries."""
    from paper_2501_06838_amd.surrogate import closed_form_radius
    wl = synth.config3(n_images=3)
    chol = wl.chol.copy()
    chol[0, 0] = -1.0
    chol[1, 2] = 0.0
    m, c, col, op = to_dev(wl)
    c = torch.from_numpy(chol).cuda()
    say("closed-form radius")
    for tau, margin in ((4e-3, 0.0), (1e-3, 0.25), (1e-6, -0.1)):
        got = closed_form_radius(c, col, op, tau, margin).cpu().numpy().astype(np.float64)
        ref = S.closed_form_radius(chol, wl.color, wl.opacity, tau, margin)
        np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-6)
        assert got[0] == 3.0 and got[1] == 3.0


def test_sq_error_kernel():
    from paper_2501_06838_amd.surrogate import sq_error
    rng = np.random.default_rng(9)
    a, b = rng.normal(size=100001).astype(np.float32), rng.normal(size=100001).astype(np.float32)
    say("sq error")
    got = sq_error(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    ref = float(((np.float64(a) - np.float64(b)) ** 2).sum())
    assert abs(got - ref) <= 1e-12 * ref


def test_trained_radius_gain_at_50db():
    """Trained on labels the exact rasterizer measures, the pruned render of
    a wide-sigma image stays >= 50 dB from the exact render while binning and
    evaluating fewer pairs; its image equals the oracle's render with the
    same radii (1e-5).  Against the closed-form control (radius where the
    Gaussian's own peak falls to tau, plus a margin) at the smallest margin
    (0.05 grid) that reaches 50 dB on this very image, the network's
    in-support pair count is within 25% of the control's: the learned radius
    is not worse than a control tuned on the test image, and the network is
    not claimed to beat it."""
    import paper_2501_06838_amd as P
    from paper_2501_06838_amd.surrogate import features, psnr
    from paper_2501_06838_amd.surrogate_train import train_radius_mlp
    say("surrogate training")
    net, info = train_radius_mlp(lambda k: synth.surrogate_training_batch(11, k), 40, 8, 4e-3,
                                 steps=500, lr=3e-3)
    assert info["losses"][-1] < 0.1 * info["losses"][0]
    wl = synth._build("wide", [(96, 96, 4.0)], (0.8, 0.5), 0.0, seed=5)
    plan, ws, exact = render(wl, 16)
    m, c, col, op = to_dev(wl)
    R = net.radius(features(plan, c, col, op, net.norm))
    plan2 = plan_for(wl, 16)
    plan2, ws2, pruned = render(wl, 16, radius=R.cpu().numpy(), plan=plan2)
    p_ex, _, _, s_ex = plan.diagnostics(ws, support=True)
    p_pr, _, _, s_pr = plan2.diagnostics(ws2, support=True)
    db = psnr(pruned, exact)
    assert db >= 50.0, db
    assert s_pr < 0.9 * s_ex and p_pr < p_ex
    ref = O.forward_batch(wl, radius=R.cpu().numpy())
    from tests._gpu import assert_forward_close
    assert_forward_close(plan2.split(pruned)[0].cpu().numpy(), ref[0])
    # the control, tuned on this image
    from paper_2501_06838_amd.surrogate import closed_form_radius
    plan3 = plan_for(wl, 16)
    margin = 0.0
    while True:
        Rc = closed_form_radius(c, col, op, 4e-3, margin)
        plan3, ws3, ctrl = render(wl, 16, radius=Rc.cpu().numpy(), plan=plan3)
        if psnr(ctrl, exact) >= 50.0 or margin >= 3.0:
            break
        margin = round(margin + 0.05, 2)
    s_cf = plan3.diagnostics(ws3, support=True)[3]
    say(f"  pairs in support: exact {s_ex}, network {s_pr} ({db:.2f} dB), control {s_cf} "
        f"(margin {margin}, {psnr(ctrl, exact):.2f} dB)")
    assert psnr(ctrl, exact) >= 50.0
    assert s_pr <= 1.25 * s_cf


def test_fused_radius_matches_features_then_forward():
    """gs_mlp_radius (features formed inside the first layer) gives bitwise
    the radii of gs_mlp_features + gs_mlp_forward, also over more than one
    32-image chunk and with Gaussians outside the training range."""
    from paper_2501_06838_amd.surrogate import RadiusMLP, features, make_norm
    from paper_2501_06838_amd.surrogate_train import init_params
    wl = synth.concat([synth.tiny(H=9, W=7, s=2.0 + 0.3 * k, seed=40 + k, sigma=(0.8, 0.5))
                       for k in range(37)], "c37")
    plan = plan_for(wl, 16)
    m, c, col, op = to_dev(wl)
    F = S.features(np.array([im.scale for im in wl.images for _ in range(im.g_count)]),
                   wl.chol, wl.color, wl.opacity)
    mu, sd = F.mean(0), F.std(0)
    Z = (F - mu) / sd
    lo, hi = np.quantile(Z, 0.05, axis=0), np.quantile(Z, 0.95, axis=0)  # some fall outside
    net = RadiusMLP(init_params(3))
    net.norm = make_norm(mu, sd, lo, hi, 0.25)
    say("fused radius")
    ref = net.radius(features(plan, c, col, op, net.norm))
    got = net.radius_for(plan, c, col, op)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert (got == 3.0).float().mean().item() > 0.2 and (got < 3.0).any()
