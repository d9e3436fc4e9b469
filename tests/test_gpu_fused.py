"""The fused tile kernel (forward render, L1 gradient and backward render of
each tile in one pass) and the one-call training step, against the separate
entry points (bitwise) and the FP64 oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from tests._gpu import assert_forward_close, assert_grad_close, plan_for, render, say, to_dev

pytestmark = pytest.mark.gpu


def _uneven(seed=31):
    shapes = [(21, 17, 2.3), (12, 30, 6.1), (7, 9, 11.7), (26, 24, 1.6)]
    return synth._build("uneven4", shapes, (0.8, 0.5), 0.25, seed, with_target=True)


CASES = [("config1x3", lambda: synth.config1(n_images=3), 16, 0),
         ("config1x3_T8", lambda: synth.config1(n_images=3), 8, 0),
         ("config1x2_T32", lambda: synth.config1(n_images=2), 32, 0),
         ("uneven_T16_B64", _uneven, 16, 64),
         ("uneven_T16_B256_persistent", _uneven, 16, 256),
         ("config2b_T16", lambda: synth.config2b(), 16, 0)]


@pytest.mark.parametrize("name,make,tile,batch", CASES, ids=[c[0] for c in CASES])
def test_fused_matches_separate_calls(name, make, tile, batch):
    wl = make()
    flags = 1 if "persistent" in name else 0
    say("fused vs separate", name, wl.n_gauss)
    plan = plan_for(wl, tile, lds_batch=batch, flags=flags)
    m, c, col, op = to_dev(wl)
    plan.ensure_capacity(m, c)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    ws1, out1 = plan.new_workspace(), plan.new_output()
    loss1 = torch.zeros((), dtype=torch.float64, device="cuda")
    plan.forward(m, c, col, op, ws1, out1)
    g1 = plan.backward_l1(c, col, op, ws1, out1, target, loss=loss1)
    ws2, out2 = plan.new_workspace(), plan.new_output()
    loss2 = torch.zeros((), dtype=torch.float64, device="cuda")
    n = wl.n_gauss
    g2 = tuple(torch.empty(s, device="cuda") for s in [(n, 2), (n, 3), (n, 3), (n,)])
    plan.step_l1(m, c, col, op, ws2, out2, target, g2, loss=loss2)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    for a, b in zip(g1, g2):
        assert torch.equal(a, b)
    assert abs(loss1.item() - loss2.item()) <= 1e-12 * loss1.item()


def test_step_against_oracle():
    """The one-call step on an uneven batch: image within 1e-5, loss and
    gradients against the FP64 oracle (L1 sign decisions taken on the GPU's
    FP32 image on both sides)."""
    wl = _uneven(7)
    say("step vs oracle", wl.n_gauss)
    plan = plan_for(wl, 16)
    m, c, col, op = to_dev(wl)
    plan.ensure_capacity(m, c)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    ws, out = plan.new_workspace(), plan.new_output()
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    n = wl.n_gauss
    g = tuple(torch.empty(s, device="cuda") for s in [(n, 2), (n, 3), (n, 3), (n,)])
    plan.step_l1(m, c, col, op, ws, out, target, g, loss=loss)
    torch.cuda.synchronize()
    imgs = [x.cpu().numpy() for x in plan.split(out)]
    for a, r in zip(imgs, O.forward_batch(wl)):
        assert_forward_close(a, r)
    ref_loss, G = O.l1_loss_and_grad(imgs, wl.target)
    assert abs(loss.item() - ref_loss) <= 1e-12 * ref_loss
    for name, a, r in zip(("mean", "chol", "color", "opacity"), g, O.backward_batch(wl, G)):
        assert_grad_close(a.cpu().numpy(), r, name=name)


def test_loss_reduction_repeats_bitwise():
    """The loss value is reduced by several workgroups (36,864 tiles), the
    last one to finish adding the partial sums and resetting the count: three
    steps in a row and the stand-alone loss kernel give the same bits."""
    wl = synth.config2b()
    say("loss repeats", wl.n_gauss)
    plan = plan_for(wl, 16)
    m, c, col, op = to_dev(wl)
    plan.ensure_capacity(m, c)
    target = plan.pack([torch.from_numpy(t) for t in wl.target]).cuda()
    ws, out = plan.new_workspace(), plan.new_output()
    n = wl.n_gauss
    g = tuple(torch.empty(s, device="cuda") for s in [(n, 2), (n, 3), (n, 3), (n,)])
    vals = []
    for _ in range(3):
        loss = torch.zeros((), dtype=torch.float64, device="cuda")
        plan.step_l1(m, c, col, op, ws, out, target, g, loss=loss)
        torch.cuda.synchronize()
        vals.append(loss.item())
    again = torch.zeros((), dtype=torch.float64, device="cuda")
    plan.l1_loss_value(ws, again)
    torch.cuda.synchronize()
    assert vals[0] == vals[1] == vals[2]
    assert abs(again.item() - vals[0]) <= 1e-12 * vals[0]
    assert vals[0] > 0
