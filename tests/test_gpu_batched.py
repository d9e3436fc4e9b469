"""Batched uneven launches: persistent tile kernels over the longest-first
tile order, the forward's LDS batch, graph replays of a persistent step, the
autotuner, and the full serving-style batch (64 uneven images) against the
FP64 oracle.

The persistent flag, the LDS batch and the binning's sort (counting or
radix) are launch choices only: the image must be bitwise the default
launch's, and so must the gradients (the per-pair sums are reduced in a
fixed order)."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from tests._gpu import assert_forward_close, assert_grad_close, plan_for, render, say, to_dev

pytestmark = pytest.mark.gpu

PERSISTENT = 0x1
RADIX = 0x4


def _small_uneven(seed=21):
    """Four uneven images, scales from x1.5 to x11.3, 25% extra Gaussians."""
    shapes = [(20, 31, 1.5), (9, 14, 11.3), (33, 17, 4.4), (5, 6, 7.9)]
    return synth._build("small_uneven", shapes, (0.6, 0.3), 0.25, seed, with_target=True)


def _step(wl, tile, lds_batch=0, flags=0):
    """Forward + fused-L1 backward; returns (plan, ws, out, grads, loss)."""
    plan = plan_for(wl, tile, lds_batch=lds_batch, flags=flags)
    plan, ws, out = render(wl, tile, plan=plan)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    m, c, col, op = to_dev(wl)
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    grads = plan.backward_l1(c, col, op, ws, out, target, loss=loss)
    torch.cuda.synchronize()
    return plan, ws, out, grads, loss


@pytest.mark.parametrize("tile,batches", [(8, (32, 64)), (16, (64, 96, 112, 128, 256)), (32, (32, 64))])
def test_persistent_and_lds_batch_are_bitwise_launch_choices(tile, batches):
    wl = synth.config3(n_images=6, with_target=True)
    say("bitwise launch choices", tile, batches, wl.n_gauss)
    _, _, out0, g0, l0 = _step(wl, tile)
    for b in batches:
        for flags in (0, PERSISTENT, RADIX, PERSISTENT | RADIX):
            say("  batch", b, "flags", flags)
            _, _, out, g, l = _step(wl, tile, b, flags)
            assert torch.equal(out, out0), (b, flags)
            assert l.item() == l0.item()
            for a, r in zip(g, g0):
                assert torch.equal(a, r), (b, flags)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_persistent_parity_against_oracle(tile):
    """Uneven batch, persistent kernels: tile lists bit-exact, forward within
    1e-5, fused-L1 gradients within 1e-3 of the FP64 oracle."""
    wl = _small_uneven()
    say("persistent parity", tile, wl.n_gauss)
    plan, ws, out, (gm, gc, gcol, gop), loss = _step(wl, tile, 0, PERSISTENT)
    ranges, gids = plan.tile_lists(ws)
    r_ref, g_ref = O.tile_lists_batch(wl, tile, tile)
    assert np.array_equal(ranges, r_ref) and np.array_equal(gids, g_ref)
    imgs = [x.cpu().numpy() for x in plan.split(out)]
    for g, r in zip(imgs, O.forward_batch(wl)):
        assert_forward_close(g, r)
    ref_loss, G = O.l1_loss_and_grad(imgs, wl.target)
    assert abs(loss.item() - ref_loss) <= 1e-12 * ref_loss
    rm, rc, rcol, rop = O.backward_batch(wl, G)
    assert_grad_close(gm.cpu().numpy(), rm, name="mean")
    assert_grad_close(gc.cpu().numpy(), rc, name="chol")
    assert_grad_close(gcol.cpu().numpy(), rcol, name="color")
    assert_grad_close(gop.cpu().numpy(), rop, name="opacity")


def test_tile_order_is_longest_first():
    wl = synth.config3(n_images=5)
    say("tile order", wl.n_gauss)
    plan, ws, _ = render(wl, 16, plan=plan_for(wl, 16, flags=PERSISTENT))
    order, ordered = plan.tile_order(ws)
    assert ordered == 1
    assert np.array_equal(np.sort(order), np.arange(plan.n_tiles, dtype=np.uint32))
    ranges, _ = plan.tile_lists(ws)
    L = (ranges[:, 1] - ranges[:, 0])[order.astype(np.int64)]
    bucket = np.where(L < 128, L, np.minimum(255, 128 + ((L - 128) >> 4)))
    assert (np.diff(bucket) <= 0).all()
    # equal buckets keep ascending tile ids (stable order)
    same = np.diff(bucket) == 0
    assert (np.diff(order.astype(np.int64))[same] > 0).all()
    # a binning without the flag marks the order as absent
    plan2, ws2, _ = render(wl, 16)
    assert plan2.tile_order(ws2)[1] == 0


@pytest.mark.parametrize("flags", [PERSISTENT, RADIX, PERSISTENT | RADIX])
def test_persistent_graph_replays_match_default_launch(flags):
    """Several replays of a captured persistent or radix-binned step (and of
    the loss reduction's counter), with eager work in between, each give
    bitwise the default launch's image, gradients and loss."""
    import paper_2501_06838_amd as P
    wl = synth.config3(n_images=4, with_target=True)
    plan = plan_for(wl, 16, flags=flags)
    m, c, col, op = to_dev(wl)
    plan.ensure_capacity(m, c, headroom=1.25)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    n = wl.n_gauss
    ws, out = plan.new_workspace(), plan.new_output()
    grads = tuple(torch.empty(s, device="cuda") for s in [(n, 2), (n, 3), (n, 3), (n,)])
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    say("persistent graph capture", n)
    graph = P.StepGraph(plan, m, c, col, op, ws, out, target, grads, loss)
    _, _, out_ref, g_ref, l_ref = _step(wl, 16)
    for rep in range(4):
        graph.launch()
        torch.cuda.synchronize()
        say("  replay", rep)
        assert torch.equal(out, out_ref), rep
        assert loss.item() == l_ref.item()
        for a, r in zip(grads, g_ref):
            assert torch.equal(a, r), rep
        _step(wl, 8, 0, PERSISTENT)  # eager persistent work on other buffers
    graph.close()


def test_autotune_returns_fastest_and_caches(tmp_path):
    from paper_2501_06838_amd.autotune import TuneCache, candidates, tune
    wl = synth.config3(n_images=6, with_target=True)
    imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
    m, c, col, op = to_dev(wl)
    plan = plan_for(wl, 16)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    cands = [x for x in candidates() if x["tile"] in (8, 16)][:6]
    cache = TuneCache(str(tmp_path / "tune.json"))
    say("autotune", len(cands))
    res = tune(imgs, m, c, col, op, target, reps=2, warmup=1, cands=cands, cache=cache)
    assert not res["cached"] and res["config"] in cands
    assert res["ms"] == min(t["ms"] for t in res["timings"])
    assert len(res["timings"]) == len(cands)
    again = tune(imgs, m, c, col, op, target, cache=TuneCache(str(tmp_path / "tune.json")))
    assert again["cached"] and again["config"] == res["config"]


def test_config3_full_batch_persistent_is_bitwise_default():
    """The serving-style batch at full size (64 uneven images): the
    persistent longest-first launch gives bitwise the default launch's image,
    loss and gradients (the default launch is held to the oracle element by
    element in test_gpu_fullsize)."""
    wl = synth.config3(with_target=True)
    say("config3 full, persistent vs default", wl.n_gauss)
    _, _, out0, g0, l0 = _step(wl, 16)
    _, _, out1, g1, l1 = _step(wl, 16, 0, PERSISTENT)
    assert torch.equal(out1, out0)
    assert l1.item() == l0.item()
    for a, b in zip(g1, g0):
        assert torch.equal(a, b)
