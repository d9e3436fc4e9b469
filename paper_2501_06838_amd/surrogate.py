"""Learned support radius (argument marshalling over the C ABI).

A small MLP (8 -> 64 -> 64 -> 1, BF16 matrix cores, FP32 accumulation)
predicts, per Gaussian and scale, the half-width R (in standard deviations) of
the box outside which the Gaussian's own contribution alpha max(c) f stays
below a threshold tau.  Rendering with ``radius=R`` (RasterPlan.forward)
bins and evaluates fewer (tile, Gaussian) pairs; R = 3 is the exact path and
the fallback for inputs outside the training range.

Everything numeric runs in the HIP library: features, labels (from the exact
rasterizer), forward, backward, Adam, the pruned render and its squared error.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import _native as N
from .raster import RasterPlan, _ptr, _stream

N_PARAMS = 4801


class gs_mlp_norm(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_float * 8), ("sd", ctypes.c_float * 8),
                ("fmin", ctypes.c_float * 8), ("fmax", ctypes.c_float * 8),
                ("margin", ctypes.c_float), ("reserved", ctypes.c_float * 3)]


def _bind():
    L = N.lib()
    if getattr(L, "_gs_mlp_bound", False):
        return L
    vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
    normp = ctypes.POINTER(gs_mlp_norm)
    L.gs_mlp_features.argtypes = [ctypes.POINTER(N.gs_image), i32, vp, vp, vp, i64, normp, vp, vp]
    L.gs_mlp_features.restype = i32
    L.gs_mlp_forward.argtypes = [vp, vp, i64, normp, vp, vp]
    L.gs_mlp_forward.restype = i32
    L.gs_mlp_radius.argtypes = [ctypes.POINTER(N.gs_image), i32, vp, vp, vp, vp, i64, normp,
                                vp, vp]
    L.gs_mlp_radius.restype = i32
    L.gs_mlp_workspace_size.argtypes = [i64, ctypes.POINTER(ctypes.c_size_t)]
    L.gs_mlp_workspace_size.restype = i32
    L.gs_mlp_grad.argtypes = [vp, vp, vp, vp, i64, f32, vp, ctypes.c_size_t, vp, vp, vp]
    L.gs_mlp_grad.restype = i32
    L.gs_mlp_adam.argtypes = [vp, vp, vp, vp, i32, f32, vp]
    L.gs_mlp_adam.restype = i32
    L.gs_radius_stats.argtypes = [ctypes.POINTER(N.gs_config), ctypes.POINTER(N.gs_image), i32,
                                  i64, vp, ctypes.c_size_t, f32, i32, vp, vp]
    L.gs_radius_stats.restype = i32
    L.gs_sq_error.argtypes = [vp, vp, i64, vp, vp]
    L.gs_sq_error.restype = i32
    L.gs_closed_form_radius.argtypes = [vp, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp,
                                        vp]
    L.gs_closed_form_radius.restype = i32
    L._gs_mlp_bound = True
    return L


def make_norm(mu, sd, fmin=None, fmax=None, margin=0.0) -> gs_mlp_norm:
    n = gs_mlp_norm()
    for k in range(8):
        n.mu[k] = float(mu[k])
        n.sd[k] = float(sd[k])
        n.fmin[k] = float(fmin[k]) if fmin is not None else -math.inf
        n.fmax[k] = float(fmax[k]) if fmax is not None else math.inf
    n.margin = float(margin)
    return n


def features(plan: RasterPlan, chol, color, opacity, norm: Optional[gs_mlp_norm] = None,
             stream=None, out=None) -> torch.Tensor:
    """[n, 8] features (standardised when norm is given)."""
    L = _bind()
    if out is None:
        out = torch.empty(plan.n_gauss, 8, dtype=torch.float32, device=chol.device)
    N.check(L.gs_mlp_features(plan._arr, len(plan.images), _ptr(chol), _ptr(color),
                              _ptr(opacity), plan.n_gauss,
                              None if norm is None else ctypes.byref(norm), _ptr(out),
                              _stream(stream)), "mlp features")
    return out


def radius_labels(plan: RasterPlan, workspace, tau: float, capacity=None,
                  stream=None, interior_only: bool = False) -> torch.Tensor:
    """Training labels from the exact render's workspace (radius=None); with
    interior_only, -1 for Gaussians whose support box the border cuts."""
    L = _bind()
    out = torch.empty(plan.n_gauss, dtype=torch.float32, device=workspace.device)
    cfg = plan.config(capacity)
    N.check(L.gs_radius_stats(ctypes.byref(cfg), plan._arr, len(plan.images), plan.n_gauss,
                              _ptr(workspace), workspace.numel(), float(tau),
                              1 if interior_only else 0, _ptr(out), _stream(stream)),
            "radius stats")
    return out


def closed_form_radius(chol, color, opacity, tau: float, margin: float = 0.0, out=None,
                       stream=None) -> torch.Tensor:
    """The support radius without the learned part (the control): where the
    Gaussian's own peak contribution falls to tau, plus margin, capped at 3."""
    L = _bind()
    n = chol.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=chol.device)
    N.check(L.gs_closed_form_radius(_ptr(chol), _ptr(color), _ptr(opacity), n, float(tau),
                                    float(margin), _ptr(out), _stream(stream)),
            "closed-form radius")
    return out


def sq_error(a: torch.Tensor, b: torch.Tensor, stream=None) -> float:
    """sum (a - b)^2 (synchronising)."""
    L = _bind()
    acc = torch.zeros((), dtype=torch.float64, device=a.device)
    N.check(L.gs_sq_error(_ptr(a), _ptr(b), a.numel(), _ptr(acc), _stream(stream)), "sq error")
    return float(acc.item())


def psnr(test: torch.Tensor, ref: torch.Tensor, peak: float = 1.0) -> float:
    mse = sq_error(test, ref) / test.numel()
    return math.inf if mse == 0.0 else 10.0 * math.log10(peak * peak / mse)


class RadiusMLP:
    """FP32 master parameters and Adam state on the device."""

    def __init__(self, params, device="cuda"):
        p = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device)
        if p.numel() != N_PARAMS:
            raise ValueError("expected %d parameters" % N_PARAMS)
        self.params = p.contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.grad = torch.zeros_like(self.params)
        self.norm: Optional[gs_mlp_norm] = None
        self._ws = None

    def predict(self, feats, stream=None) -> torch.Tensor:
        """Raw prediction for standardised features [n, 8]."""
        L = _bind()
        out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        N.check(L.gs_mlp_forward(_ptr(self.params), _ptr(feats), feats.shape[0], None, _ptr(out),
                                 _stream(stream)), "mlp forward")
        return out

    def radius(self, feats, stream=None, out=None) -> torch.Tensor:
        """Support half-width for the pruned path (needs self.norm)."""
        L = _bind()
        if self.norm is None:
            raise RuntimeError("calibrate the network first")
        if out is None:
            out = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
        N.check(L.gs_mlp_forward(_ptr(self.params), _ptr(feats), feats.shape[0],
                                 ctypes.byref(self.norm), _ptr(out), _stream(stream)),
                "mlp radius")
        return out

    def radius_for(self, plan: RasterPlan, chol, color, opacity, out=None, stream=None):
        """Support half-widths of a batch's Gaussians in one kernel (features
        formed inside the network's first layer; needs self.norm)."""
        L = _bind()
        if self.norm is None:
            raise RuntimeError("calibrate the network first")
        if out is None:
            out = torch.empty(plan.n_gauss, dtype=torch.float32, device=chol.device)
        N.check(L.gs_mlp_radius(plan._arr, len(plan.images), _ptr(self.params), _ptr(chol),
                                _ptr(color), _ptr(opacity), plan.n_gauss,
                                ctypes.byref(self.norm), _ptr(out), _stream(stream)),
                "mlp radius (fused)")
        return out

    def _workspace(self, n, device):
        L = _bind()
        b = ctypes.c_size_t()
        N.check(L.gs_mlp_workspace_size(n, ctypes.byref(b)), "mlp workspace")
        if self._ws is None or self._ws.numel() < b.value:
            self._ws = torch.empty(b.value, dtype=torch.uint8, device=device)
        return self._ws

    def gradient(self, feats, labels=None, dout=None, quantile=0.9, loss=None, stream=None):
        """Fills self.grad (pinball loss on labels, or upstream gradient dout)."""
        L = _bind()
        n = feats.shape[0]
        ws = self._workspace(n, feats.device)
        N.check(L.gs_mlp_grad(_ptr(self.params), _ptr(feats), _ptr(labels), _ptr(dout), n,
                              float(quantile), _ptr(ws), ws.numel(), _ptr(self.grad), _ptr(loss),
                              _stream(stream)), "mlp grad")
        return self.grad

    def step(self, feats, labels, lr=1e-3, quantile=0.9, loss=None, stream=None):
        """One training step: gradient of the pinball loss, then Adam."""
        L = _bind()
        self.gradient(feats, labels, quantile=quantile, loss=loss, stream=stream)
        self.t += 1
        N.check(L.gs_mlp_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(self.grad),
                              self.t, float(lr), _stream(stream)), "mlp adam")

    # -- persistence (weights, Adam state, normalisation) ---------------------
    def save(self, path):
        nm = self.norm
        np.savez(path, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(), t=self.t,
                 norm=np.array([] if nm is None else
                               list(nm.mu) + list(nm.sd) + list(nm.fmin) + list(nm.fmax) +
                               [nm.margin], dtype=np.float64))

    @classmethod
    def load(cls, path, device="cuda"):
        z = np.load(path, allow_pickle=False)
        net = cls(z["params"], device)
        net.m.copy_(torch.from_numpy(z["m"]))
        net.v.copy_(torch.from_numpy(z["v"]))
        net.t = int(z["t"])
        nm = z["norm"]
        if nm.size:
            net.norm = make_norm(nm[0:8], nm[8:16], nm[16:24], nm[24:32], nm[32])
        return net
