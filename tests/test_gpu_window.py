"""Algorithm 1's r-window support (rasterization ratio r, Sec. 3.1 "Fast
Rasterization") on the GPU against the FP64 oracle: tile lists bit-exact,
images within 1e-5 per element, gradients within the gradient tolerance;
small cases whole, the paper-shaped 720x720 workloads whole at x8 and
sampled at x4."""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from tests._gpu import assert_forward_close, assert_grad_close, plan_for, say, to_dev

pytestmark = pytest.mark.gpu

RADIX = 0x4
THREADS = max(1, min(16, os.cpu_count() or 1))


def _grid_workload(H, W, s, grid, seed, n_images=1):
    """Images of grid^2 Gaussians per LR pixel with L1 targets."""
    parts, images, targets, begin = [], [], [], 0
    for k in range(n_images):
        rng = np.random.default_rng([seed, k])
        m, c, col, op = synth.draw_grid_gaussians(rng, H + k, W + 2 * k, grid, 0.5, 0.4)
        parts.append((m, c, col, op))
        images.append(synth.Image(H + k, W + 2 * k, s, begin, m.shape[0]))
        begin += m.shape[0]
        oh, ow = O.output_size(H + k, W + 2 * k, s)
        targets.append(np.random.default_rng([seed, k, 1]).uniform(0, 1, (3, oh, ow))
                       .astype(np.float32))
    cat = lambda j: np.concatenate([p[j] for p in parts])
    return synth.Workload("grid", images, cat(0), cat(1), cat(2), cat(3), targets)


def _step(wl, r, flags=0, tile=16):
    plan = plan_for(wl, tile, flags=flags, window=r)
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


@pytest.mark.parametrize("r,s,tile,flags", [(0.1, 3.0, 16, 0), (0.25, 2.5, 8, 0),
                                            (0.1, 4.0, 32, RADIX), (0.05, 6.0, 16, RADIX)])
def test_window_step_against_oracle(r, s, tile, flags):
    wl = _grid_workload(24, 20, s, 2, seed=31, n_images=2)
    say("window step", r, s, tile, flags, "n", wl.n_gauss)
    plan, ws, out, grads, loss = _step(wl, r, flags, tile)
    npairs, overflow, n_invalid, n_support = plan.diagnostics(ws, support=True)
    assert overflow == 0 and n_invalid == 0
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, tile, tile, window=r)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    assert n_support == O.support_pairs_batch(wl, window=r)
    imgs = [x.cpu().numpy() for x in plan.split(out)]
    for g, ref in zip(imgs, O.forward_batch(wl, threads=THREADS, window=r)):
        assert_forward_close(g, ref)
    ref_loss, G = O.l1_loss_and_grad(imgs, wl.target)
    assert abs(loss.item() - ref_loss) <= 1e-12 * ref_loss
    ref = O.backward_batch(wl, G, threads=THREADS, window=r)
    for name, a, b in zip(("mean", "chol", "color", "opacity"), grads, ref):
        assert_grad_close(a.cpu().numpy(), b, name=name)


def test_window_rejects_a_radius_array():
    from paper_2501_06838_amd import _native as N
    wl = _grid_workload(8, 8, 2.0, 1, seed=32)
    plan = plan_for(wl, 16, window=0.1)
    m, c, col, op = to_dev(wl)
    rad = torch.full((wl.n_gauss,), 2.0, device="cuda")
    with pytest.raises(N.GSError):
        plan.count_pairs(m, c, rad)


def test_paper720_x8_whole_against_oracle():
    """720x720 at x8: 90x90 LR, 129,600 Gaussians, r = 0.1 (a 143 to 144
    pixel window each): every list, pixel and gradient."""
    wl = synth.paper720(8, seed=0, with_target=True)
    say("paper720 x8", wl.n_gauss)
    plan, ws, out, grads, loss = _step(wl, 0.1)
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, 16, 16, window=0.1)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    img = plan.split(out)[0].cpu().numpy()
    say("  oracle forward, threads", THREADS)
    ref = O.forward_batch(wl, threads=THREADS, window=0.1)[0]
    assert_forward_close(img, ref)
    _, G = O.l1_loss_and_grad([img], wl.target)
    say("  oracle backward")
    ref_g = O.backward_batch(wl, G, threads=THREADS, window=0.1)
    for name, a, b in zip(("mean", "chol", "color", "opacity"), grads, ref_g):
        assert_grad_close(a.cpu().numpy(), b, name=name)


def test_paper720_x4_sampled_against_oracle():
    """720x720 at x4: 180x180 LR, 518,400 Gaussians, r = 0.1: lists whole,
    4,000 sampled pixels, and 1,500 sampled Gaussians' gradients."""
    wl = synth.paper720(4, seed=1, with_target=True)
    say("paper720 x4", wl.n_gauss)
    plan, ws, out, grads, loss = _step(wl, 0.1)
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, 16, 16, window=0.1)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    img = plan.split(out)[0].cpu().numpy()
    rng = np.random.default_rng(33)
    xs, ys = rng.integers(0, 720, 4000), rng.integers(0, 720, 4000)
    ref = O.pixel_values(180, 180, 4.0, wl.mean, wl.chol, wl.color, wl.opacity, xs, ys,
                         window=0.1)
    assert_forward_close(img[:, ys, xs], ref)
    # gradients of a sample of Gaussians for the upstream gradient of the
    # GPU's own image (the backward treats each Gaussian independently)
    _, G = O.l1_loss_and_grad([img], wl.target)
    pick = np.sort(rng.choice(wl.n_gauss, 1500, replace=False))
    sub = [a[pick] for a in (wl.mean, wl.chol, wl.color, wl.opacity)]
    ref_g = O.backward(180, 180, 4.0, *sub, G[0], threads=THREADS, window=0.1)
    full = [a.cpu().numpy() for a in grads]
    for name, a, b in zip(("mean", "chol", "color", "opacity"), full, ref_g):
        # the tolerance's floor is relative to the largest gradient of all
        scale = np.abs(a).max()
        err = np.abs(a[pick].astype(np.float64) - b)
        assert (err <= 1e-3 * np.abs(b) + 1e-5 * scale).all(), name
