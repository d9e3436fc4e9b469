"""Launch-configuration autotuner for a batch layout (host orchestration only).

The tunable knobs of the library are the HR tile side, the number of
Gaussians the forward stages in LDS per round (``lds_batch``), whether the
tile kernels run persistent over the longest-first tile order
(``GS_FLAG_PERSISTENT``) and the binning (per-tile counting with a list sort,
or the device radix sort, ``GS_FLAG_RADIX_SORT``).  None of them changes the
rendered image (the forward sums every pixel's Gaussians in ascending index
whatever the tile and batch, and both binnings give the same lists), and the
gradients are bitwise independent of the batch, the binning and the
persistent flag.

``tune`` times one whole training step (binning, the fused tile kernel:
render, L1 gradient and backward, then the gradients) of the caller's own
batch for each candidate with HIP events on the current stream and returns
the fastest; results are cached in a JSON file keyed by the batch layout,
the device and the timing mode, so a serving loop pays the search once per
layout.  By default the step is timed as a captured HIP graph replay, as a
serving loop runs it: eager launches add a per-kernel launch cost that
favours the binning with fewer kernels (on a 2048 x 2048 render the radix
sort is the slower binning eagerly and the faster one replayed).
"""
from __future__ import annotations

import hashlib
import json
import os
import statistics
from typing import Dict, List, Optional, Sequence, Tuple

from . import _native as N

# (tile, lds_batch) pairs the library accepts
TILE_BATCHES: Tuple[Tuple[int, int], ...] = ((8, 32), (8, 64), (16, 64), (16, 96), (16, 112),
                                             (16, 128), (16, 256), (32, 32), (32, 64))


# the library's own default launch (tile 16, its default LDS batch, one
# workgroup per tile), kept unless a candidate is clearly faster
DEFAULT_LAUNCH: Dict[str, int] = {"tile": 16, "lds_batch": 96, "flags": 0}


def pick(timings: List[dict], margin: float = 0.02) -> dict:
    """The fastest timing entry, except that the default launch stays when
    no candidate beats it by more than `margin` (a fraction of its time):
    candidates within timing noise of each other do not flip the choice."""
    best = min(timings, key=lambda t: t["ms"])
    dflt = next((t for t in timings if t["config"] == DEFAULT_LAUNCH), None)
    if dflt is not None and best["ms"] > dflt["ms"] * (1.0 - margin):
        return dflt
    return best


def candidates(persistent: Sequence[bool] = (False, True),
               radix: Sequence[bool] = (False, True)) -> List[Dict[str, int]]:
    out = []
    for tile, batch in TILE_BATCHES:
        for r in radix:
            for p in persistent:
                out.append({"tile": tile, "lds_batch": batch,
                            "flags": (N.GS_FLAG_PERSISTENT if p else 0) |
                                     (N.GS_FLAG_RADIX_SORT if r else 0)})
    return out


def layout_key(images: Sequence[Tuple[int, int, float, int, int]], device_name: str,
               mode: str = "graph") -> str:
    """Cache key: the images' LR sizes, scales and Gaussian counts, the
    device, the timing mode and the library ABI version."""
    desc = [(int(h), int(w), float(s), int(gc)) for (h, w, s, _gb, gc) in images]
    blob = json.dumps({"images": desc, "device": device_name, "mode": mode,
                       "abi": int(N.lib().gs_abi_version())}, sort_keys=True)
    return hashlib.sha1(blob.encode()).hexdigest()


def default_cache_path() -> str:
    return os.environ.get("GS_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsraster",
                                       "autotune.json"))


class TuneCache:
    """JSON file {key: {"config": {...}, "ms": float, "timings": [...]}}."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or default_cache_path()
        self.entries: Dict[str, dict] = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    data = json.load(f)
                if isinstance(data, dict):
                    self.entries = data
            except (OSError, ValueError):
                self.entries = {}

    def get(self, key: str) -> Optional[dict]:
        e = self.entries.get(key)
        if not isinstance(e, dict) or "config" not in e:
            return None
        c = e["config"]
        if (int(c.get("tile", 0)), int(c.get("lds_batch", 0))) not in TILE_BATCHES:
            return None
        return e

    def put(self, key: str, entry: dict) -> None:
        self.entries[key] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def time_step(plan, mean, chol, color, opacity, target, reps: int = 3, warmup: int = 1,
              headroom: float = 1.0, captured: bool = True) -> Tuple[float, int]:
    """Median milliseconds of one training step for plan's config (a replay
    of the step captured as a HIP graph, or with `captured` False an eager
    gs_raster_step_l1), and its pair count."""
    import torch
    from .raster import StepGraph
    dev = mean.device
    n = plan.n_gauss
    pairs = plan.ensure_capacity(mean, chol, headroom=headroom)
    ws = plan.new_workspace(dev)
    out = plan.new_output(dev)
    grads = (torch.empty(n, 2, device=dev), torch.empty(n, 3, device=dev),
             torch.empty(n, 3, device=dev), torch.empty(n, device=dev))
    stream = torch.cuda.current_stream()

    graph = None
    if captured:
        graph = StepGraph(plan, mean, chol, color, opacity, ws, out, target, grads)

    def step():
        if graph is not None:
            graph.launch()
        else:
            plan.step_l1(mean, chol, color, opacity, ws, out, target, grads)

    for _ in range(warmup):
        step()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step()
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    if graph is not None:
        graph.close()
    if plan.diagnostics(ws)[1]:
        raise N.GSError(N.GS_E_CAPACITY, "autotune step")
    del ws, out, grads
    return statistics.median(times), pairs


def tune(images: Sequence[Tuple[int, int, float, int, int]], mean, chol, color, opacity,
         target, reps: int = 3, warmup: int = 1,
         cands: Optional[List[Dict[str, int]]] = None, cache: Optional[TuneCache] = None,
         force: bool = False, log=None, margin: float = 0.02, captured: bool = True) -> dict:
    """Fastest configuration for this batch (see `pick`): {"config": {tile,
    lds_batch, flags}, "ms": ..., "timings": [...], "cached": bool}."""
    import torch
    from .raster import RasterPlan
    name = torch.cuda.get_device_name(mean.device)
    key = layout_key(images, name, "graph" if captured else "eager")
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return dict(hit, cached=True)
    timings = []
    for c in (cands if cands is not None else candidates()):
        plan = RasterPlan(images, mean.shape[0], tile=c["tile"], lds_batch=c["lds_batch"],
                          flags=c["flags"])
        ms, pairs = time_step(plan, mean, chol, color, opacity, target, reps, warmup,
                              captured=captured)
        timings.append({"config": dict(c), "ms": round(ms, 5), "pairs": pairs})
        if log:
            log(f"autotune {c}: {ms:.4f} ms, {pairs} pairs")
    best = pick(timings, margin)
    entry = {"config": best["config"], "ms": best["ms"], "timings": timings, "device": name}
    if cache is not None:
        cache.put(key, entry)
    return dict(entry, cached=False)
