"""The alternative readings of Eq. 4 and of the truncation on the GPU against
the FP64 oracle: pixel-centre sampling (GS_FLAG_PIXEL_CENTER: HR pixel x
samples u = (x + 1/2)/s - 1/2) and the elliptical support (GS_FLAG_ELLIPSE:
Mahalanobis distance below R inside the box), alone and together.

Both sides decide support membership with the same FP64 operation sequence,
so tile lists and in-support pair counts must match bit for bit; images are
held to 1e-5 per element (with exact zeros where the oracle's are) and
gradients to the gradient tolerance, as for the literal reading."""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from tests._gpu import assert_forward_close, assert_grad_close, plan_for, say, to_dev

pytestmark = pytest.mark.gpu

PC, EL = 0x8, 0x10
PERSISTENT, ATOMIC, RADIX = 0x1, 0x2, 0x4
THREADS = max(1, min(16, os.cpu_count() or 1))


def _oracle_mode(flags):
    return (O.PIXEL_CENTER if flags & PC else 0) | (O.ELLIPSE if flags & EL else 0)


def _workload(seed):
    """Three uneven images (ragged tiles at every tile size) with L1 targets."""
    parts = [synth.tiny(H=23, W=19, s=3.7, seed=seed, sigma=(0.7, 0.4), extra_frac=0.3,
                        with_target=True),
             synth.tiny(H=9, W=31, s=2.2, seed=seed + 1, sigma=(0.6, 0.3), with_target=True),
             synth.tiny(H=12, W=12, s=5.5, seed=seed + 2, sigma=(0.9, 0.5), extra_frac=0.2,
                        with_target=True)]
    return synth.concat(parts, name="modes")


def _step(wl, tile, flags):
    plan = plan_for(wl, tile, flags=flags)
    m, c, col, op = to_dev(wl)
    plan.ensure_capacity(m, c)
    ws, out = plan.new_workspace(), plan.new_output()
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    n = wl.n_gauss
    grads = tuple(torch.empty(sh, device="cuda") for sh in [(n, 2), (n, 3), (n, 3), (n,)])
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    plan.step_l1(m, c, col, op, ws, out, target, grads, loss=loss)
    torch.cuda.synchronize()
    return plan, ws, out, grads, loss


@pytest.mark.parametrize("mode,tile,extra", [(PC, 16, 0), (EL, 16, 0), (PC | EL, 16, 0),
                                             (PC, 8, RADIX), (EL, 8, RADIX),
                                             (PC | EL, 32, PERSISTENT),
                                             (EL, 16, PERSISTENT | ATOMIC)])
def test_mode_step_against_oracle(mode, tile, extra):
    wl = _workload(seed=51)
    om = _oracle_mode(mode)
    say("mode step", hex(mode), "tile", tile, "flags", hex(extra), "n", wl.n_gauss)
    plan, ws, out, grads, loss = _step(wl, tile, mode | extra)
    npairs, overflow, n_invalid, n_support = plan.diagnostics(ws, support=True)
    assert overflow == 0 and n_invalid == 0
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, tile, tile, mode=om)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    assert n_support == O.support_pairs_batch(wl, mode=om)
    imgs = [x.cpu().numpy() for x in plan.split(out)]
    for g, ref in zip(imgs, O.forward_batch(wl, threads=THREADS, mode=om)):
        assert_forward_close(g, ref)
    ref_loss, G = O.l1_loss_and_grad(imgs, wl.target)
    assert abs(loss.item() - ref_loss) <= 1e-12 * ref_loss
    ref = O.backward_batch(wl, G, threads=THREADS, mode=om)
    for name, a, b in zip(("mean", "chol", "color", "opacity"), grads, ref):
        assert_grad_close(a.cpu().numpy(), b, name=name)


def test_ellipse_drops_pixels_and_pixel_centre_moves_them():
    """Against the literal reading on the same Gaussians: the ellipse keeps
    the same tile lists (they follow the box) but fewer in-support pairs; the
    pixel-centre convention moves the image."""
    wl = _workload(seed=52)
    plan0, ws0, out0, _, _ = _step(wl, 16, 0)
    plan1, ws1, out1, _, _ = _step(wl, 16, EL)
    plan2, ws2, out2, _, _ = _step(wl, 16, PC)
    r0, g0 = plan0.tile_lists(ws0)
    r1, g1 = plan1.tile_lists(ws1)
    assert np.array_equal(r0, r1) and np.array_equal(g0, g1)
    s0 = plan0.diagnostics(ws0, support=True)[3]
    s1 = plan1.diagnostics(ws1, support=True)[3]
    assert 0 < s1 < s0
    assert (out1 <= out0).all()  # non-negative colours and opacities: a subset of terms
    assert not torch.equal(out0, out2)


def test_mode_config0_whole():
    """48x48 LR at x4 (192x192, 2,304 Gaussians), both readings together:
    every list, pixel and gradient."""
    wl = synth.config0(seed=3, with_target=True)
    om = O.PIXEL_CENTER | O.ELLIPSE
    say("config0 pixel-centre + ellipse", wl.n_gauss)
    plan, ws, out, grads, loss = _step(wl, 16, PC | EL)
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, 16, 16, mode=om)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    img = plan.split(out)[0].cpu().numpy()
    assert_forward_close(img, O.forward_batch(wl, threads=THREADS, mode=om)[0])
    _, G = O.l1_loss_and_grad([img], wl.target)
    ref = O.backward_batch(wl, G, threads=THREADS, mode=om)
    for name, a, b in zip(("mean", "chol", "color", "opacity"), grads, ref):
        assert_grad_close(a.cpu().numpy(), b, name=name)


def test_config2a_ellipse_sampled():
    """2048x2048 from 512x512 LR (262,144 Gaussians) with both readings:
    lists whole, 4,000 sampled pixels, and 1,500 sampled Gaussians' gradients
    for the upstream gradient of the GPU's own image."""
    wl = synth.config2a(seed=4)
    om = O.PIXEL_CENTER | O.ELLIPSE
    say("config2a pixel-centre + ellipse", wl.n_gauss)
    plan, ws, out, grads, loss = _step(wl, 16, PC | EL)
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, 16, 16, mode=om)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    img = plan.split(out)[0].cpu().numpy()
    rng = np.random.default_rng(53)
    xs, ys = rng.integers(0, 2048, 4000), rng.integers(0, 2048, 4000)
    ref = O.pixel_values(512, 512, 4.0, wl.mean, wl.chol, wl.color, wl.opacity, xs, ys,
                         mode=om)
    assert_forward_close(img[:, ys, xs], ref)
    _, G = O.l1_loss_and_grad([img], wl.target)
    pick = np.sort(rng.choice(wl.n_gauss, 1500, replace=False))
    sub = [a[pick] for a in (wl.mean, wl.chol, wl.color, wl.opacity)]
    ref_g = O.backward(512, 512, 4.0, *sub, G[0], threads=THREADS, mode=om)
    full = [a.cpu().numpy() for a in grads]
    for name, a, b in zip(("mean", "chol", "color", "opacity"), full, ref_g):
        scale = np.abs(a).max()
        err = np.abs(a[pick].astype(np.float64) - b)
        assert (err <= 1e-3 * np.abs(b) + 1e-5 * scale).all(), name
