"""PyTorch face of the gfx950 rasterizer (argument marshalling only).

Every step of the render runs in the HIP library behind include/gs_raster.h;
PyTorch only supplies device memory, the current stream and autograd.

    plan = RasterPlan([(H, W, s, g_begin, g_count), ...], n_gauss, tile=16)
    out = rasterize(mean, chol, color, opacity, plan)     # flat, differentiable
    images = plan.split(out)                              # [3, out_h, out_w] views

Gaussians are packed image after image: image k owns entries
[g_begin, g_begin + g_count).  Parameters (paper Sec. 3.1): mean (mu_x, mu_y)
in LR pixels, covariance as its Cholesky factor (l11, l21, l22), peak colour c,
opacity alpha.  The HR image of an H x W input at scale s has
floor(sH + 0.5) x floor(sW + 0.5) pixels, sampled at (x/s, y/s) (Eq. 4).
"""
from __future__ import annotations

import ctypes
import math
from typing import List, Optional, Sequence, Tuple

import torch

from . import _native as N

__all__ = ["RasterPlan", "GSRasterize", "StepGraph", "rasterize", "l1_loss_grad"]


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_param(t: torch.Tensor, name: str, shape) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class RasterPlan:
    """A validated batch layout: HR sizes, packed output offsets, workspace
    sizing and direct calls of the C ABI.

    images: sequence of (lr_h, lr_w, scale, g_begin, g_count).
    tile:   HR tile side (8, 16 or 32).
    window: 0 for the standard-deviation support box; r > 0 for Algorithm 1's
            r-window (rasterization ratio r).
    """

    def __init__(self, images: Sequence[Tuple[int, int, float, int, int]], n_gauss: int,
                 tile: int = 16, lds_batch: int = 0, flags: int = 0,
                 pair_capacity: int = 0, window: float = 0.0):
        if len(images) < 1:
            raise ValueError("need at least one image")
        self.n_gauss = int(n_gauss)
        self.tile = int(tile)
        self.lds_batch = int(lds_batch)
        self.flags = int(flags)
        self.window = float(window)
        self.sizes: List[Tuple[int, int]] = []
        self.offsets: List[int] = []
        arr = (N.gs_image * len(images))()
        off = 0
        for k, (h, w, s, gb, gc) in enumerate(images):
            oh, ow = ctypes.c_int32(), ctypes.c_int32()
            N.check(N.lib().gs_output_size(int(h), int(w), float(s), ctypes.byref(oh),
                                           ctypes.byref(ow)), f"image {k} size")
            self.sizes.append((oh.value, ow.value))
            self.offsets.append(off)
            arr[k] = N.gs_image(int(h), int(w), float(s), int(gb), int(gc), off)
            off += 3 * oh.value * ow.value
        self.images = list(images)
        self.out_numel = off
        self._arr = arr
        self.capacity = int(pair_capacity)
        self._cfg_cache = None
        self.workspace_bytes(1)  # validates the layout now

    # -- configuration --------------------------------------------------------
    def config(self, capacity: Optional[int] = None) -> N.gs_config:
        cap = self.capacity if capacity is None else int(capacity)
        return N.gs_config(self.tile, self.lds_batch, self.flags, 0, cap, self.window)

    def workspace_bytes(self, capacity: Optional[int] = None) -> int:
        cfg = self.config(max(1, self.capacity if capacity is None else capacity))
        b = ctypes.c_size_t()
        N.check(N.lib().gs_workspace_size(ctypes.byref(cfg), self._arr, len(self.images),
                                          self.n_gauss, ctypes.byref(b)), "workspace size")
        return b.value

    @property
    def n_tiles(self) -> int:
        t = self.tile
        return sum(((w + t - 1) // t) * ((h + t - 1) // t) for h, w in self.sizes)

    def new_workspace(self, device="cuda", capacity: Optional[int] = None) -> torch.Tensor:
        return torch.empty(self.workspace_bytes(capacity), dtype=torch.uint8, device=device)

    def new_output(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.out_numel, dtype=torch.float32, device=device)

    def split(self, flat: torch.Tensor) -> List[torch.Tensor]:
        """Per-image [3, out_h, out_w] views of a packed output or gradient."""
        out = []
        for (oh, ow), off in zip(self.sizes, self.offsets):
            out.append(flat[off:off + 3 * oh * ow].view(3, oh, ow))
        return out

    def pack(self, images: Sequence[torch.Tensor]) -> torch.Tensor:
        return torch.cat([im.reshape(-1) for im in images])

    # -- direct ABI calls -----------------------------------------------------
    def count_pairs(self, mean, chol, radius=None, stream=None) -> int:
        """Exact number of (tile, Gaussian) pairs (synchronising)."""
        n = self.n_gauss
        _check_param(mean, "mean", (n, 2))
        _check_param(chol, "chol", (n, 3))
        ws = torch.empty(self.workspace_bytes(1), dtype=torch.uint8, device=mean.device)
        cfg = self.config(1)
        p = ctypes.c_int64()
        N.check(N.lib().gs_count_pairs(ctypes.byref(cfg), self._arr, len(self.images),
                                       _ptr(mean), _ptr(chol), _ptr(radius), n, _ptr(ws),
                                       ws.numel(), ctypes.byref(p), _stream(stream)),
                "count pairs")
        return p.value

    def ensure_capacity(self, mean, chol, radius=None, headroom: float = 1.0) -> int:
        """Sizes the pair capacity from the exact count (synchronising)."""
        need = self.count_pairs(mean, chol, radius)
        if need > self.capacity or self.capacity <= 0:
            self.capacity = max(1, int(math.ceil(need * headroom)))
        return need

    def forward(self, mean, chol, color, opacity, workspace, out, radius=None, stream=None,
                capacity=None):
        n = self.n_gauss
        _check_param(mean, "mean", (n, 2))
        _check_param(chol, "chol", (n, 3))
        _check_param(color, "color", (n, 3))
        _check_param(opacity, "opacity", (n,))
        if radius is not None:
            _check_param(radius, "radius", (n,))
        _check_param(out, "out", (self.out_numel,))
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_forward(ctypes.byref(cfg), self._arr, len(self.images),
                                          _ptr(mean), _ptr(chol), _ptr(color), _ptr(opacity),
                                          _ptr(radius), n, _ptr(workspace), workspace.numel(),
                                          _ptr(out), _stream(stream)), "forward")

    def backward(self, mean, chol, color, opacity, workspace, grad_out, grads=None,
                 radius=None, stream=None, capacity=None):
        n = self.n_gauss
        _check_param(grad_out, "grad_out", (self.out_numel,))
        if grads is None:
            dev = grad_out.device
            grads = (torch.empty(n, 2, device=dev), torch.empty(n, 3, device=dev),
                     torch.empty(n, 3, device=dev), torch.empty(n, device=dev))
        gm, gc, gcol, gop = grads
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_backward(ctypes.byref(cfg), self._arr, len(self.images),
                                           _ptr(mean), _ptr(chol), _ptr(color),
                                           _ptr(opacity), _ptr(radius), n, _ptr(workspace),
                                           workspace.numel(), _ptr(grad_out), _ptr(gm),
                                           _ptr(gc), _ptr(gcol), _ptr(gop), _stream(stream)),
                "backward")
        return grads

    # -- the four stages, one C call each (used by timing code) -------------
    def bin(self, mean, chol, color, opacity, workspace, radius=None, stream=None,
            capacity=None):
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_bin(ctypes.byref(cfg), self._arr, len(self.images),
                                      _ptr(mean), _ptr(chol), _ptr(color), _ptr(opacity),
                                      _ptr(radius), self.n_gauss, _ptr(workspace),
                                      workspace.numel(), _stream(stream)), "bin")

    def render(self, workspace, out, stream=None, capacity=None):
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_render(ctypes.byref(cfg), self._arr, len(self.images),
                                         self.n_gauss, _ptr(workspace), workspace.numel(),
                                         _ptr(out), _stream(stream)), "render")

    def render_backward(self, workspace, grad_out, stream=None, capacity=None):
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_render_backward(ctypes.byref(cfg), self._arr,
                                                  len(self.images), self.n_gauss,
                                                  _ptr(workspace), workspace.numel(),
                                                  _ptr(grad_out), _stream(stream)),
                "render backward")

    def render_backward_l1(self, workspace, out, target, stream=None, capacity=None):
        """Backward render for the L1 loss against `target` (fused gradient)."""
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_render_backward_l1(ctypes.byref(cfg), self._arr,
                                                     len(self.images), self.n_gauss,
                                                     _ptr(workspace), workspace.numel(),
                                                     _ptr(out), _ptr(target), _stream(stream)),
                "render backward l1")

    def render_fused_l1(self, workspace, out, target, stream=None, capacity=None):
        """Forward render into out, L1 gradient against target and backward
        render, per tile in one kernel (workspace from bin())."""
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_render_fused_l1(ctypes.byref(cfg), self._arr, len(self.images),
                                                  self.n_gauss, _ptr(workspace),
                                                  workspace.numel(), _ptr(out), _ptr(target),
                                                  _stream(stream)), "render fused l1")

    def step_l1(self, mean, chol, color, opacity, workspace, out, target, grads, loss=None,
                radius=None, stream=None, capacity=None):
        """One training step of the L1 loss: binning, fused render, gradients
        (overwritten into grads = (mean, chol, color, opacity)) and, when
        given, the mean loss into loss (device double)."""
        cfg = self.config(capacity)
        gm, gc, gcol, gop = grads
        N.check(N.lib().gs_raster_step_l1(ctypes.byref(cfg), self._arr, len(self.images),
                                          _ptr(mean), _ptr(chol), _ptr(color), _ptr(opacity),
                                          _ptr(radius), self.n_gauss, _ptr(workspace),
                                          workspace.numel(), _ptr(out), _ptr(target), _ptr(gm),
                                          _ptr(gc), _ptr(gcol), _ptr(gop), _ptr(loss),
                                          _stream(stream)), "step l1")

    def step_l1_noalloc(self, mean, chol, color, opacity, out, target, grads, loss=None,
                        radius=None, overflow=None, stream=None):
        """step_l1 on the library's own device scratch array (no workspace, no
        device allocation).  overflow: optional int32 device tensor [1] set to
        1 if the pairs exceeded the capacity that fits the array."""
        cfg = self.config(self.capacity)
        gm, gc, gcol, gop = grads
        N.check(N.lib().gs_raster_step_l1_noalloc(
            ctypes.byref(cfg), self._arr, len(self.images), _ptr(mean), _ptr(chol),
            _ptr(color), _ptr(opacity), _ptr(radius), self.n_gauss, _ptr(out), _ptr(target),
            _ptr(gm), _ptr(gc), _ptr(gcol), _ptr(gop), _ptr(loss), _ptr(overflow),
            _stream(stream)), "step l1 (no allocation)")

    def l1_loss_value(self, workspace, loss, stream=None, capacity=None):
        """Mean L1 loss of the last fused backward into `loss` (0-d float64 tensor)."""
        cfg = self.config(capacity)
        N.check(N.lib().gs_l1_loss_value(ctypes.byref(cfg), self._arr, len(self.images),
                                         self.n_gauss, _ptr(workspace), workspace.numel(),
                                         _ptr(loss), _stream(stream)), "l1 loss value")

    def backward_l1(self, chol, color, opacity, workspace, out, target, grads=None, loss=None,
                    stream=None, capacity=None):
        """Training-step backward for the L1 loss: gradients (and the loss)."""
        n = self.n_gauss
        _check_param(out, "out", (self.out_numel,))
        _check_param(target, "target", (self.out_numel,))
        if grads is None:
            dev = out.device
            grads = (torch.empty(n, 2, device=dev), torch.empty(n, 3, device=dev),
                     torch.empty(n, 3, device=dev), torch.empty(n, device=dev))
        gm, gc, gcol, gop = grads
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_backward_l1(ctypes.byref(cfg), self._arr, len(self.images),
                                              _ptr(chol), _ptr(color), _ptr(opacity), n,
                                              _ptr(workspace), workspace.numel(), _ptr(out),
                                              _ptr(target), _ptr(gm), _ptr(gc), _ptr(gcol),
                                              _ptr(gop), _ptr(loss), _stream(stream)),
                "backward l1")
        return grads

    def gradients(self, chol, color, opacity, workspace, grads, stream=None, capacity=None):
        gm, gc, gcol, gop = grads
        cfg = self.config(capacity)
        N.check(N.lib().gs_raster_gradients(ctypes.byref(cfg), self._arr, len(self.images),
                                            _ptr(chol), _ptr(color), _ptr(opacity),
                                            self.n_gauss, _ptr(workspace), workspace.numel(),
                                            _ptr(gm), _ptr(gc), _ptr(gcol), _ptr(gop),
                                            _stream(stream)), "gradients")

    def diagnostics(self, workspace, stream=None, capacity=None, support=False):
        """(n_pairs, overflow, n_invalid[, n_support]) of the last forward
        (synchronising).  n_support = in-support (pixel, Gaussian) pairs."""
        cfg = self.config(capacity)
        p, o, inv, sup = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        st = N.lib().gs_diagnostics(ctypes.byref(cfg), self._arr, len(self.images),
                                    self.n_gauss, _ptr(workspace), workspace.numel(),
                                    ctypes.byref(p), ctypes.byref(o), ctypes.byref(inv),
                                    ctypes.byref(sup), _stream(stream))
        if st not in (N.GS_OK, N.GS_E_CAPACITY):
            N.check(st, "diagnostics")
        if support:
            return p.value, o.value, inv.value, sup.value
        return p.value, o.value, inv.value

    def tile_lists(self, workspace, stream=None, capacity=None):
        """(ranges [tiles, 2] int32, gids [P] int32) of the last forward."""
        import numpy as np
        cfg = self.config(capacity)
        nt, npairs = ctypes.c_int64(), ctypes.c_int64()
        N.check(N.lib().gs_tile_lists(ctypes.byref(cfg), self._arr, len(self.images),
                                      self.n_gauss, _ptr(workspace), workspace.numel(),
                                      None, None, 0, ctypes.byref(nt), ctypes.byref(npairs),
                                      _stream(stream)), "tile lists (sizes)")
        ranges = np.zeros((nt.value, 2), dtype=np.int32)
        gids = np.zeros(max(1, npairs.value), dtype=np.int32)
        N.check(N.lib().gs_tile_lists(ctypes.byref(cfg), self._arr, len(self.images),
                                      self.n_gauss, _ptr(workspace), workspace.numel(),
                                      ranges.ctypes.data_as(ctypes.c_void_p),
                                      gids.ctypes.data_as(ctypes.c_void_p), gids.size,
                                      ctypes.byref(nt), ctypes.byref(npairs),
                                      _stream(stream)), "tile lists")
        return ranges, gids[:npairs.value]


    def tile_order(self, workspace, stream=None, capacity=None):
        """(order [n_tiles] uint32, ordered flag) of the persistent kernels."""
        import numpy as np
        cfg = self.config(capacity)
        order = np.zeros(self.n_tiles, dtype=np.uint32)
        flag = ctypes.c_int32()
        N.check(N.lib().gs_tile_order(ctypes.byref(cfg), self._arr, len(self.images),
                                      self.n_gauss, _ptr(workspace), workspace.numel(),
                                      order.ctypes.data_as(ctypes.c_void_p), order.size,
                                      ctypes.byref(flag), _stream(stream)), "tile order")
        return order, flag.value


class StepGraph:
    """A captured HIP graph of one forward (+ fused L1 backward) pass over a
    plan's batch with fixed buffers; ``launch()`` replays it on the current
    stream.  Update the Gaussian tensors in place between replays."""

    def __init__(self, plan: "RasterPlan", mean, chol, color, opacity, workspace, out,
                 target=None, grads=None, loss=None, radius=None, capacity=None):
        self.plan = plan
        # keep every buffer alive as long as the graph
        self.buffers = (mean, chol, color, opacity, workspace, out, target, grads, loss, radius)
        cfg = plan.config(capacity)
        gm = gc = gcol = gop = None
        if grads is not None:
            gm, gc, gcol, gop = grads
        h = ctypes.c_void_p()
        N.check(N.lib().gs_graph_create(ctypes.byref(cfg), plan._arr, len(plan.images),
                                        _ptr(mean), _ptr(chol), _ptr(color), _ptr(opacity),
                                        _ptr(radius), plan.n_gauss, _ptr(workspace),
                                        workspace.numel(), _ptr(out), _ptr(target), _ptr(gm),
                                        _ptr(gc), _ptr(gcol), _ptr(gop), _ptr(loss),
                                        ctypes.byref(h)), "graph create")
        self._h = h

    def launch(self, stream=None):
        N.check(N.lib().gs_graph_launch(self._h, _stream(stream)), "graph launch")

    def close(self):
        if self._h:
            N.lib().gs_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GSRasterize(torch.autograd.Function):
    """Differentiable batch render: out = render(mean, chol, color, opacity).

    The forward's workspace (render records, sorted pair lists, tile ranges)
    is saved for the backward.  If the pair capacity of the plan is too small
    the forward sizes it exactly and renders again (``check=True``)."""

    @staticmethod
    def forward(ctx, mean, chol, color, opacity, plan: RasterPlan, radius=None,
                check: bool = True):
        if plan.capacity <= 0:
            plan.ensure_capacity(mean, chol, radius)
        cap = plan.capacity
        ws = plan.new_workspace(mean.device, cap)
        out = plan.new_output(mean.device)
        plan.forward(mean, chol, color, opacity, ws, out, radius, capacity=cap)
        if check:
            npairs, overflow, _ = plan.diagnostics(ws, capacity=cap)
            if overflow:
                cap = plan.capacity = max(plan.capacity, npairs)
                ws = plan.new_workspace(mean.device, cap)
                plan.forward(mean, chol, color, opacity, ws, out, radius, capacity=cap)
        ctx.plan = plan
        ctx.radius = radius
        ctx.capacity = cap
        ctx.save_for_backward(mean, chol, color, opacity, ws)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        mean, chol, color, opacity, ws = ctx.saved_tensors
        gm, gc, gcol, gop = ctx.plan.backward(mean, chol, color, opacity, ws,
                                              grad_out.contiguous(), radius=ctx.radius,
                                              capacity=ctx.capacity)
        return gm, gc, gcol, gop, None, None, None


def rasterize(mean, chol, color, opacity, plan: RasterPlan, radius=None, check=True):
    """Packed HR images of the batch (flat float32), differentiable."""
    return GSRasterize.apply(mean, chol, color, opacity, plan, radius, check)


def l1_loss_grad(img: torch.Tensor, target: torch.Tensor, stream=None):
    """(mean |img - target| as a 0-d float64 tensor, d loss / d img)."""
    _check_param(img, "img", tuple(img.shape))
    _check_param(target, "target", tuple(img.shape))
    grad = torch.empty_like(img)
    loss = torch.empty((), dtype=torch.float64, device=img.device)
    N.check(N.lib().gs_l1_loss_grad(_ptr(img), _ptr(target), img.numel(), _ptr(grad),
                                    _ptr(loss), _stream(stream)), "l1 loss")
    return loss, grad
