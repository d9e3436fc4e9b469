"""Helpers shared by the GPU parity tests (inputs to the device, tolerances)."""
import sys

import numpy as np
import torch

import paper_2501_06838_amd as G


def say(*a):
    """Names the case before each GPU step (flushed, so a crash still shows it)."""
    print("[case]", *a, file=sys.stderr, flush=True)


def to_dev(wl, device="cuda"):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return t(wl.mean), t(wl.chol), t(wl.color), t(wl.opacity)


def plan_for(wl, tile=16, **kw):
    imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
    return G.RasterPlan(imgs, wl.n_gauss, tile=tile, **kw)


def render(wl, tile=16, radius=None, plan=None):
    """Forward through the C ABI; returns (plan, workspace, flat image)."""
    plan = plan or plan_for(wl, tile)
    m, c, col, op = to_dev(wl)
    rad = None if radius is None else torch.from_numpy(np.float32(radius)).cuda()
    plan.ensure_capacity(m, c, rad)
    ws = plan.new_workspace()
    out = plan.new_output()
    plan.forward(m, c, col, op, ws, out, rad)
    torch.cuda.synchronize()
    return plan, ws, out


def assert_forward_close(got, ref, rtol=1e-5, floor=1e-30):
    """Element-wise |got - ref| <= rtol |ref| (+ a floor far below FP32's
    normal range); exact zeros where the reference is exactly zero."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape
    err = np.abs(got - ref)
    bad = err > rtol * np.abs(ref) + floor
    assert not bad.any(), (
        f"{bad.sum()} elements off; worst rel "
        f"{(err / np.maximum(np.abs(ref), 1e-300)).max():.3e}")
    assert (got[ref == 0] == 0).all()
    return float((err / np.maximum(np.abs(ref), 1e-300))[ref != 0].max(initial=0.0))


def assert_grad_close(got, ref, rtol=1e-3, name=""):
    """Per tensor: |g - r| <= rtol |r| + 1e-5 max|r| element-wise and
    max|g - r| / max|r| <= rtol."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    assert (err <= rtol * np.abs(ref) + 1e-5 * scale).all(), (
        f"{name}: worst {(err / (np.abs(ref) + 1e-5 * scale + 1e-300)).max():.3e}")
    assert err.max() <= rtol * scale, f"{name}: inf-norm rel {err.max() / scale:.3e}"
    return float(err.max() / max(scale, 1e-300))
