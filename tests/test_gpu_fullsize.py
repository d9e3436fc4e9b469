"""Full-size training steps against the FP64 oracle, element by element.

The DIV2K-sized single renders (2048^2 at x4, 3072^2 at x12, wide sigmas)
and the serving-style batch (64 uneven images, x1.5 to x12), each run as the
benchmark runs them (gs_raster_step_l1, tile 16, default LDS batch): tile
lists bit-exact, every pixel of every image within 1e-5, the L1 loss, and
every gradient of every Gaussian within the gradient tolerance.  The L1
gradient's sign is taken on the GPU's FP32 image on both sides.  The
radix-sort binning (three 8-bit passes over the tile ids of the 64-image
batch) must reproduce the lists, the image and the gradients bit for bit.
The oracle runs its OpenMP variants (bitwise its serial results).
"""
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


def _step(wl, flags):
    plan = plan_for(wl, 16, flags=flags)
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


@pytest.mark.parametrize("which", ["config2a", "config2b", "config3"])
def test_full_size_step_against_oracle(which):
    wl = synth.by_name(which, with_target=True)
    say("full size", which, "n", wl.n_gauss, "counting binning")
    plan, ws, out, grads, loss = _step(wl, 0)
    npairs, overflow, n_invalid, n_support = plan.diagnostics(ws, support=True)
    assert overflow == 0 and n_invalid == 0
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, 16, 16)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    assert npairs == len(g_ref)
    assert n_support == O.support_pairs_batch(wl)

    imgs = [x.cpu().numpy() for x in plan.split(out)]
    say("  oracle forward, threads", THREADS)
    for g, r in zip(imgs, O.forward_batch(wl, threads=THREADS)):
        assert_forward_close(g, r)
    ref_loss, G = O.l1_loss_and_grad(imgs, wl.target)
    assert abs(loss.item() - ref_loss) <= 1e-12 * ref_loss
    say("  oracle backward")
    ref = O.backward_batch(wl, G, threads=THREADS)
    del G
    for name, a, r in zip(("mean", "chol", "color", "opacity"), grads, ref):
        assert_grad_close(a.cpu().numpy(), r, name=name)

    say("  radix binning")
    plan_r, ws_r, out_r, grads_r, loss_r = _step(wl, RADIX)
    if which == "config3":
        assert plan_r.n_tiles > 1 << 16  # three 8-bit passes over the tile ids
    ranges_r, gids_r = plan_r.tile_lists(ws_r)
    assert np.array_equal(ranges_r, r_ref) and np.array_equal(gids_r, g_ref)
    assert torch.equal(out_r, out)
    assert loss_r.item() == loss.item()
    for a, b in zip(grads_r, grads):
        assert torch.equal(a, b)
