"""The allocation-free training step (gs_raster_step_l1_noalloc: its
workspace is the library's own device array) against gs_raster_step_l1 with a
caller workspace, through the C ABI: image, loss and every gradient bit for
bit, on two calls in a row, the second with a smaller batch (whatever the
first left in the shared array must not leak into the second)."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_2501_06838_amd import _native as N
from paper_2501_06838_amd.raster import _ptr, _stream
from tests._gpu import plan_for, say, to_dev

pytestmark = pytest.mark.gpu


def _buffers(plan, n):
    nan = float("nan")
    out = torch.full((plan.out_numel,), nan, device="cuda")
    grads = [torch.full(sh, nan, device="cuda") for sh in [(n, 2), (n, 3), (n, 3), (n,)]]
    loss = torch.full((), nan, dtype=torch.float64, device="cuda")
    return out, grads, loss


def _step(wl, noalloc):
    plan = plan_for(wl, 16)
    m, c, col, op = to_dev(wl)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    out, grads, loss = _buffers(plan, wl.n_gauss)
    flag = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    if noalloc:
        cfg = N.gs_config(16, 0, 0, 0, 0)  # capacity: the largest that fits the array
        N.check(N.lib().gs_raster_step_l1_noalloc(
            ctypes.byref(cfg), plan._arr, len(plan.images), _ptr(m), _ptr(c), _ptr(col),
            _ptr(op), None, wl.n_gauss, _ptr(out), _ptr(target), *[_ptr(g) for g in grads],
            _ptr(loss), _ptr(flag), _stream()), "no-alloc step")
    else:
        plan.ensure_capacity(m, c)
        ws = plan.new_workspace()
        plan.step_l1(m, c, col, op, ws, out, target, grads, loss=loss)
    torch.cuda.synchronize()
    return out, grads, loss, int(flag.item())


def test_noalloc_step_matches_workspace_step_twice():
    big = synth.config1()                                   # 16 x 237^2, 65,536 Gaussians
    small = synth.tiny(H=20, W=17, s=2.7, seed=5, n_images=3, with_target=True)
    for name, wl in (("config1", big), ("3 x 20x17 at 2.7", small)):
        say("no-alloc step", name, "n", wl.n_gauss)
        got = _step(wl, noalloc=True)
        ref = _step(wl, noalloc=False)
        assert got[3] == 0  # no pair overflow
        assert torch.equal(got[0], ref[0]), "image"
        for a, b in zip(got[1], ref[1]):
            assert torch.equal(a, b), "gradient"
        assert got[2].item() == ref[2].item(), "loss"
        assert np.isfinite(got[2].item())
