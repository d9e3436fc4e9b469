"""Throughput of the scale-aware 2D Gaussian rasterizer on one MI355X.

One step = one training pass of the whole hot path over the workload's
batch: support boxes, tile binning (pair counting and per-tile list sort),
tile ranges, the fused tile kernel (forward render, L1 gradient against the
target, backward render) and the per-Gaussian gradients with the loss value,
every kernel from the HIP library, the step captured as one HIP graph and
replayed.  Inputs are resident in HBM before timing starts.

Headline workload (the metric's configuration): one 512x512 LR image with
262,144 seeded synthetic Gaussians (wide sigmas), rendered at s = 4 to
2048x2048, exact 3-sigma support, L1 loss to a seeded uniform target.  The
same JSON line carries the surrogate-pruned comparison at >= 50 dB on that
workload and on 256x256 -> 3072x3072 at s = 12, the other workloads with
their roofline fractions, the 64-image batch, and the FP64 oracle timed on
the host's cores.

    python bench.py [--steps K] [--warmup W] [--workload config2a]

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "HR megapixels/s fwd+bwd (exact vs surrogate-pruned at ≥50 dB); % of roofline"

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 64 lanes x 2 (FMA) x 2 (packed)
PEAK_HBM_GBS = 8000.0

# Algorithmic work per in-support (HR pixel, Gaussian) pair, in FP32
# FLOP-equivalents at the packed-FP32 issue rate (one exp2 at quarter rate
# occupies the slots of 16 FLOP): forward 16 FLOP + 1 exp = 32,
# backward 32 FLOP + 1 exp = 48.
FLOPEQ_FWD = 32.0
FLOPEQ_BWD = 48.0
# Algorithmic HBM bytes: 24 per HR pixel (12 B image written by the forward,
# 12 B target read for the L1 gradient) and 108 per Gaussian (36 B read by
# the forward, 36 B by the backward, 36 B of gradients written).
BYTES_PER_PX = 24.0
BYTES_PER_GAUSS = 108.0

# Counter readings of k_render_fused on config2a per launch configuration
# (rocprofv3 --pmc runs, FETCH_SIZE then WRITE_SIZE, KiB per dispatch
# averaged; summaries and commands in
# profiles/config2a_k_render_fused_traffic.md), valid while the render
# sources hash to `sources` (otherwise reported as null).  The factors scale
# FETCH_SIZE and WRITE_SIZE by what the counters read for a plain 256 MiB
# device copy.
PROFILE = {"workload": "config2a", "sources": "0fd317bab16fbe6d",
           "launches": {
               (16, 96, 0): {"fetch_kib": 41152.2, "write_kib": 164374.8},
               (16, 112, 0): {"fetch_kib": 37853.5, "write_kib": 95029.3},
               (16, 128, 0): {"fetch_kib": 37822.1, "write_kib": 95012.4}},
           "fetch_factor": 2.313, "write_factor": 1.157}
PROFILE_SOURCES = ("paper_2501_06838_amd/csrc/gs_render.hip",
                   "paper_2501_06838_amd/csrc/gs_internal.h")

WORKLOADS = {
    "config0": "48x48 LR (2,304 Gaussians) -> 192x192 at s=4, fwd+bwd, L1 loss",
    "config1": "16 x 64x64 LR (4,096 Gaussians each) -> 237x237 at s=3.7, fwd+bwd, L1 loss",
    "config2a": "512x512 LR (262,144 Gaussians) -> 2048x2048 at s=4, fwd+bwd, L1 loss",
    "config2b": "256x256 LR (65,536 Gaussians) -> 3072x3072 at s=12, fwd+bwd, L1 loss",
    "config3": "64 uneven images, LR U{48..256}^2 +25% Gaussians, s~U[1.5,12], fwd+bwd, "
               "L1 loss",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def render_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in PROFILE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_entry(workload, launch):
    P = PROFILE
    if P["sources"] is None or workload != P["workload"] or render_sources_hash() != P["sources"]:
        return None
    return P["launches"].get((launch["tile"], launch["lds_batch"], launch["flags"]))


def traffic_bytes(workload, launch):
    e = profile_entry(workload, launch)
    if e is None:
        return None
    return round(e["fetch_kib"] * 1024 * PROFILE["fetch_factor"] +
                 e["write_kib"] * 1024 * PROFILE["write_factor"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def host_threads():
    """Cores this process may run on (its share of the host), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, seconds: float):
    """The FP64 C oracle on whole images of the same workload, round-robin
    until `seconds` have elapsed: forward, L1 gradient, backward.  Once on one
    thread and once on all the host's threads (the oracle's OpenMP variants:
    row bands for the forward, Gaussians for the backward; same arithmetic,
    bitwise the same results)."""
    import numpy as np
    from oracle import oracle as O
    O.lib()

    def run(threads):
        t0 = time.perf_counter()
        px = n = k = 0
        while True:
            i = k % len(wl.images)
            im, sl = wl.images[i], wl.image_slice(i)
            img = O.forward(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl], wl.color[sl],
                            wl.opacity[sl], threads=threads)
            g = np.sign(img - wl.target[i]) / img.size
            O.backward(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl], wl.color[sl],
                       wl.opacity[sl], g, threads=threads)
            px += img.shape[1] * img.shape[2]
            n += 1
            k += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return px / el / 1e6, n, px, el

    nt = host_threads()
    v1, n1, px1, el1 = run(1)
    vn, nn, pxn, eln = run(nt)
    what = "FP64 C oracle, forward + L1 gradient + backward"
    return {
        "value": round(vn, 4), "unit": "HR megapixels/s", "cores": nt, "kind": "oracle",
        "sample": f"{nn} whole images of the workload ({pxn} HR px) in {eln:.1f} s on {nt} "
                  f"threads: {what}",
        "one_core": {"value": round(v1, 4), "cores": 1,
                     "sample": f"{n1} whole images ({px1} HR px) in {el1:.1f} s, one thread"},
        "cpu": cpu_model(), "host_cpus": os.cpu_count(),
    }


class Bench:
    """Device-resident inputs of one workload and helpers to time its step."""

    def __init__(self, G, synth, torch, np, name, seed=0, wl=None, window=0.0):
        self.G, self.torch, self.np = G, torch, np
        self.dev = torch.device("cuda:0")
        self.name = name
        self.window = window
        self.wl = wl if wl is not None else synth.by_name(name, seed=seed, with_target=True)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.dev)
        wl = self.wl
        self.mean, self.chol, self.color, self.opacity = (t(wl.mean), t(wl.chol), t(wl.color),
                                                          t(wl.opacity))
        self.imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
        self.n = wl.n_gauss
        self.target = G.RasterPlan(self.imgs, self.n).pack([t(x) for x in wl.target])
        self.host_target = wl.target

    def buffers(self, plan):
        torch, dev, n = self.torch, self.dev, self.n
        ws, out = plan.new_workspace(dev), plan.new_output(dev)
        grads = (torch.empty(n, 2, device=dev), torch.empty(n, 3, device=dev),
                 torch.empty(n, 3, device=dev), torch.empty(n, device=dev))
        loss = torch.zeros((), dtype=torch.float64, device=dev)
        return ws, out, grads, loss

    def plan(self, launch, radius=None, headroom=1.0):
        plan = self.G.RasterPlan(self.imgs, self.n, window=self.window, **launch)
        pairs = plan.ensure_capacity(self.mean, self.chol, radius, headroom=headroom)
        return plan, pairs


def warm_up(torch, launch_fn, min_launches, seconds):
    """At least min_launches untimed launches, continued until `seconds` of
    back-to-back work have run: the GPU's clocks ramp up under sustained load
    (a cold start measured 10-15% slow on the first brackets), so every timed
    region follows continuous work."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while n < min_launches or time.perf_counter() - t0 < seconds:
        for _ in range(8):
            launch_fn()
        n += 8
        torch.cuda.synchronize()


def time_graph(torch, launch_fn, reps, brackets=3):
    """Median over `brackets` of the mean milliseconds per replay of reps
    back-to-back replays (wall clock, synchronised on both sides)."""
    res = []
    for _ in range(brackets):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            launch_fn()
        torch.cuda.synchronize()
        res.append((time.perf_counter() - t0) * 1e3 / reps)
    return statistics.median(res), res


def kernel_ms(torch, stream, fn, reps):
    """Average milliseconds of one launch of fn over reps back-to-back
    launches, bracketed by HIP events on the stream the kernel runs on."""
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def tile_kernel_times(B, plan, ws, out, reps):
    """(fused, forward, backward) tile-kernel milliseconds on a binned batch."""
    torch = B.torch
    stream = torch.cuda.current_stream()
    plan.bin(B.mean, B.chol, B.color, B.opacity, ws)
    # one untimed launch of each kernel first: a kernel's first launch in a
    # process may load its code object
    plan.render_fused_l1(ws, out, B.target)
    plan.render(ws, out)
    plan.render_backward_l1(ws, out, B.target)
    plan.render_fused_l1(ws, out, B.target)
    torch.cuda.synchronize()
    fused = kernel_ms(torch, stream, lambda: plan.render_fused_l1(ws, out, B.target), reps)
    fwd = kernel_ms(torch, stream, lambda: plan.render(ws, out), reps)
    bwd = kernel_ms(torch, stream, lambda: plan.render_backward_l1(ws, out, B.target), reps)
    return fused, fwd, bwd


def valu_probe(torch, blocks=4096, iters=4096):
    """The library's vector-ALU probe (gs_valu_probe, compiled like the tile
    kernels: packed FP32 off): FMA rate, exp2 rate, the render-shaped mix
    (five FMA-class operations and one exp2 per step), and the issue cost of
    three lane-mask forms next to one FMA per step (a select on an SGPR-pair
    mask, a select on a mask read with readfirstlane, a one-bit field
    extract ANDed into the value), as SIMD cycles per wave64 step taking
    the FMA-only step as 4 cycles; each from HIP events around launches of
    `blocks` workgroups after an untimed launch."""
    from paper_2501_06838_amd import _native as N
    from paper_2501_06838_amd.raster import _ptr, _stream
    out = torch.empty(blocks * 256, device="cuda")
    L = N.lib()
    stream = torch.cuda.current_stream()
    steps = float(blocks) * 256 * iters * 8  # lane-steps per launch (8 chains)
    res = {"blocks": blocks, "threads": 256, "iters": iters, "chains": 8}
    ms = {}
    for kind in range(6):
        def fn(k=kind):
            N.check(L.gs_valu_probe(k, blocks, iters, _ptr(out), _stream()), "valu probe")
        fn()
        ms[kind] = kernel_ms(torch, stream, fn, 3)
        rate = steps / (ms[kind] * 1e-3)
        if kind == 0:
            res["fma_tflops"] = round(2 * rate / 1e12, 2)
        elif kind == 1:
            res["exp2_per_s"] = round(rate, -9)
        elif kind == 2:
            res["mix_steps_per_s"] = round(rate, -9)
    res["mask_step_cycles"] = {
        "fma_only": 4.0,
        "fma_select_sgpr_mask": round(4.0 * ms[3] / ms[0], 2),
        "fma_readfirstlane_mask_select": round(4.0 * ms[4] / ms[0], 2),
        "fma_bit_extract_and": round(4.0 * ms[5] / ms[0], 2)}
    return res


def roofline_fracs(n_support, hr_px, n_gauss, step_ms, fused_ms):
    """T_roof / T_measured end to end (the step) and render-only (the fused
    tile kernel), T_roof = max(VALU, HBM) time of the algorithmic work."""
    t_valu = n_support * (FLOPEQ_FWD + FLOPEQ_BWD) / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
    t_hbm = (hr_px * BYTES_PER_PX + n_gauss * BYTES_PER_GAUSS) / (PEAK_HBM_GBS * 1e9)
    t_roof = max(t_valu, t_hbm)
    return {"t_roof_us": round(t_roof * 1e6, 2),
            "bound": "alu" if t_valu >= t_hbm else "hbm",
            "end_to_end": round(t_roof / (step_ms * 1e-3), 4),
            "render_only": round(t_roof / (fused_ms * 1e-3), 4)}


def step_record(B, launch, reps, kernels=True):
    """Captured step of one workload: median of three brackets of reps
    replays, tile-kernel times and roofline fractions."""
    G, torch = B.G, B.torch
    plan, pairs = B.plan(launch)
    ws, out, grads, loss = B.buffers(plan)
    plan.step_l1(B.mean, B.chol, B.color, B.opacity, ws, out, B.target, grads, loss=loss)
    torch.cuda.synchronize()
    npairs, overflow, n_invalid, n_support = plan.diagnostics(ws, support=True)
    if overflow:
        raise SystemExit(f"pair capacity overflow ({B.name})")
    graph = G.StepGraph(plan, B.mean, B.chol, B.color, B.opacity, ws, out, B.target, grads,
                        loss)
    warm_up(torch, graph.launch, 3, 0.05)
    ms, brackets = time_graph(torch, graph.launch, reps)
    if plan.diagnostics(ws)[1]:
        raise SystemExit(f"pair capacity overflow during replay ({B.name})")
    graph.close()
    hr_px = plan.out_numel // 3
    rec = {"workload": f"{B.name}: {WORKLOADS.get(B.name, B.name)}", "ms_per_step": round(ms, 5),
           "brackets_ms": [round(x, 5) for x in brackets], "replays_per_bracket": reps,
           "mp_s": round(hr_px / (ms * 1e-3) / 1e6, 2), "hr_pixels": hr_px,
           "gaussians": B.n, "tile_pairs": npairs, "support_pairs": n_support,
           "launch_config": launch}
    if kernels:
        fused, fwd, bwd = tile_kernel_times(B, plan, ws, out, reps)
        rec["fused_kernel_us"] = round(fused * 1e3, 2)
        if B.window > 0.0:
            rec["roofline_frac"] = None
            rec["window_pairs_per_s"] = round(n_support / (fused * 1e-3), 1)
        else:
            rec["roofline_frac"] = roofline_fracs(n_support, hr_px, B.n, ms, fused)
    del ws, out, grads
    return rec


def autotune(B, reps=5):
    from paper_2501_06838_amd.autotune import tune
    t0 = time.perf_counter()
    res = tune(B.imgs, B.mean, B.chol, B.color, B.opacity, B.target, reps=reps, warmup=2)
    timings = [[c["config"]["tile"], c["config"]["lds_batch"], c["config"]["flags"], c["ms"]]
               for c in res["timings"]]
    return res["config"], timings, time.perf_counter() - t0


def batched_uneven(G, synth, torch, np, reps):
    """The serving-style batch: 64 uneven images rendered fwd+bwd in one
    captured step, with the launch picked by the autotuner; the default
    launch and the persistent longest-first launch are timed beside it
    (median of three brackets of reps replays each)."""
    log("batched: config3 (64 uneven images)")
    B = Bench(G, synth, torch, np, "config3")
    best, timings, t_tune = autotune(B)
    log(f"batched: autotuner picked {best} in {t_tune:.1f} s")
    out = {"workload": "config3: " + WORKLOADS["config3"], "images": len(B.imgs),
           "autotune": {"config": best, "seconds": round(t_tune, 2), "timings_ms": timings}}
    launches = {"tuned": best, "default_launch": {"tile": 16, "lds_batch": 96, "flags": 0},
                "persistent_lpt": {"tile": 16, "lds_batch": 96,
                                   "flags": G.GS_FLAG_PERSISTENT}}
    done = {}
    for name, cfg in launches.items():
        key = json.dumps(cfg, sort_keys=True)
        if key in done:  # the same launch is timed once
            out[name] = {"same_as": done[key]}
            continue
        out[name] = step_record(B, cfg, reps, kernels=True)
        done[key] = name
    out["launch"] = "each step captured as one HIP graph, replayed"
    return out


def forward_record(B, launch, reps):
    """Captured forward-only pass (binning + tile render) of one workload:
    median of three brackets of reps replays, and the forward tile kernel's
    HIP-event time."""
    torch = B.torch
    plan, _ = B.plan(launch)
    ws, out = plan.new_workspace(B.dev), plan.new_output(B.dev)
    graph = B.G.StepGraph(plan, B.mean, B.chol, B.color, B.opacity, ws, out)
    warm_up(torch, graph.launch, 3, 0.05)
    ms, brackets = time_graph(torch, graph.launch, reps)
    if plan.diagnostics(ws)[1]:
        raise SystemExit(f"pair capacity overflow ({B.name})")
    graph.close()
    npairs, _, _, n_support = plan.diagnostics(ws, support=True)
    stream = torch.cuda.current_stream()
    plan.render(ws, out)  # untimed first launch
    fwd = kernel_ms(torch, stream, lambda: plan.render(ws, out), reps)
    hr_px = plan.out_numel // 3
    del ws, out
    rec = {"ms_per_pass": round(ms, 5), "brackets_ms": [round(x, 5) for x in brackets],
           "mp_s": round(hr_px / (ms * 1e-3) / 1e6, 2), "tile_pairs": npairs,
           "support_pairs": n_support, "fwd_kernel_us": round(fwd * 1e3, 2),
           "launch_config": launch}
    if B.window > 0.0:
        # Algorithm 1's window pairs per second; most of them lie where the
        # Gaussian's weight underflows and are never evaluated (the kernels
        # drop such blocks at staging), so no ALU roofline fraction is
        # formed on this count
        rec["window_pairs_per_s"] = round(n_support / (fwd * 1e-3), 1)
    else:
        tf = n_support * FLOPEQ_FWD / (fwd * 1e-3) / 1e12
        rec["fwd_kernel_tflops"] = round(tf, 3)
        rec["fwd_kernel_frac"] = round(tf / PEAK_FP32_VECTOR_TFLOPS, 4)
    return rec


# The paper's render-only forward times on an A100 (supplement, "Rendering
# Cost Comparison", 720x720 GT, r = 0.1): context, another machine.
PAPER_RENDER_MS = {4: 168.0, 8: 71.0}


def paper_window(G, synth, torch, np, scales, reps):
    """Algorithm 1's r-window (r = 0.1) on the paper's cost workload (720x720
    output, m = 16 Gaussians per LR pixel): the forward-only pass the paper
    times, and the fwd+bwd training step, each captured as one graph."""
    out = []
    for s in scales:
        wl = synth.paper720(s, seed=0, with_target=True)
        log(f"paper720 x{s}: {wl.n_gauss} Gaussians, r = 0.1")
        B = Bench(G, synth, torch, np, f"paper720_x{s}", wl=wl, window=0.1)
        # both binnings: the window's lists are long (tens of thousands of
        # Gaussians per tile), where the radix sort overtakes the per-tile
        # list sort; the faster is reported, the other kept beside it
        fwds = {f: forward_record(B, {"tile": 16, "lds_batch": 96, "flags": f}, reps)
                for f in (0, G.GS_FLAG_RADIX_SORT)}
        best = min(fwds, key=lambda f: fwds[f]["ms_per_pass"])
        fwd = fwds[best]
        step = step_record(B, {"tile": 16, "lds_batch": 96, "flags": best}, reps)
        rec = {"workload": f"paper720_x{s}: {wl.images[0].lr_h}x{wl.images[0].lr_w} LR, "
                           f"{wl.n_gauss} Gaussians (16 per LR pixel) -> 720x720 at s={s}, "
                           f"r-window r = 0.1",
               "forward": fwd, "fwd_bwd_step": step,
               "forward_other_binning": fwds[G.GS_FLAG_RADIX_SORT if best == 0 else 0]}
        if s in PAPER_RENDER_MS:
            rec["paper_render_ms_a100"] = PAPER_RENDER_MS[s]
            rec["forward_vs_paper_render"] = round(PAPER_RENDER_MS[s] / fwd["ms_per_pass"], 1)
        log(f"  forward {fwd['ms_per_pass']} ms, fwd+bwd {step['ms_per_step']} ms "
            f"(paper's A100 render: {PAPER_RENDER_MS.get(s)} ms)")
        out.append(rec)
        del B
    return out


def head_and_psnr(G, synth, torch, np, reps):
    """The Gaussian primary head (forward + backward) on the paper's x4
    workload size (518,400 Gaussians) and the Y-channel PSNR of two
    2048x2048 renders: HIP-event times against the HBM peak."""
    from paper_2501_06838_amd.head import head_images, psnr_y
    from paper_2501_06838_amd import _native as N
    from paper_2501_06838_amd.raster import _ptr, _stream
    import ctypes
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    grid, H = 4, 180
    images = head_images([(H, H)], grid)
    n = images[0][3]
    g = torch.Generator(device=dev).manual_seed(5)
    raw = [torch.randn(sh, device=dev, generator=g) for sh in [(n,), (n, 3), (n, 2), (n,),
                                                               (n, 2)]]
    outs = [torch.empty(sh, device=dev) for sh in [(n, 2), (n, 3), (n, 3), (n,)]]
    grads = [torch.randn(sh, device=dev, generator=g) for sh in [(n, 2), (n, 3), (n, 3), (n,)]]
    d = [torch.empty(sh, device=dev) for sh in [(n,), (n, 3), (n, 2), (n,), (n, 2)]]
    arr = (N.gs_image * 1)(N.gs_image(H, H, 1.0, 0, n, 0))
    L = N.lib()

    def fwd():
        N.check(L.gs_gaussian_head_forward(arr, 1, grid, *[_ptr(t) for t in raw], n,
                                           *[_ptr(t) for t in outs], _stream()), "head")

    def bwd():
        N.check(L.gs_gaussian_head_backward(n, *[_ptr(t) for t in raw[:4]],
                                            *[_ptr(t) for t in grads], *[_ptr(t) for t in d],
                                            _stream()), "head bwd")
    fwd(), bwd()
    f_ms = kernel_ms(torch, stream, fwd, reps)
    b_ms = kernel_ms(torch, stream, bwd, reps)
    f_bytes, b_bytes = 72.0 * n, 100.0 * n
    head = {"gaussians": n, "grid": grid,
            "forward": {"us": round(f_ms * 1e3, 2), "bytes": f_bytes,
                        "gb_s": round(f_bytes / (f_ms * 1e-3) / 1e9, 1),
                        "frac_hbm": round(f_bytes / (f_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
            "backward": {"us": round(b_ms * 1e3, 2), "bytes": b_bytes,
                         "gb_s": round(b_bytes / (b_ms * 1e-3) / 1e9, 1),
                         "frac_hbm": round(b_bytes / (b_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}}
    del raw, outs, grads, d
    plan = G.RasterPlan([(512, 512, 4.0, 0, 0)], 0)
    a = torch.rand(plan.out_numel, device=dev, generator=g)
    b = (a + 0.01 * torch.randn(plan.out_numel, device=dev, generator=g)).contiguous()
    psnr_y(plan, a, b)
    p_ms = kernel_ms(torch, stream, lambda: psnr_y(plan, a, b), reps)
    p_bytes = 24.0 * plan.out_numel // 3
    p, _ = psnr_y(plan, a, b)
    ps = {"hr_pixels": plan.out_numel // 3, "us": round(p_ms * 1e3, 2), "psnr_db": round(p.item(), 3),
          "bytes": p_bytes, "gb_s": round(p_bytes / (p_ms * 1e-3) / 1e9, 1),
          "frac_hbm": round(p_bytes / (p_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
          "note": "three launches per call (clear, sums, PSNR)"}
    log(f"head fwd {head['forward']['gb_s']} GB/s, bwd {head['backward']['gb_s']} GB/s; "
        f"psnr_y {ps['gb_s']} GB/s")
    return {"gaussian_head": head, "psnr_y_2048": ps}


def calibrate_control(G, synth, torch, np, tau, target_db=50.5):
    """Margin of the closed-form radius control so that its pruned render
    reaches target_db PSNR against the exact render on held-out images of
    the config-2 distribution (seeds and sizes distinct from the measured
    workloads): the smallest margin on a 0.05 grid that reaches it on all."""
    from paper_2501_06838_amd.surrogate import closed_form_radius, psnr
    dev = torch.device("cuda:0")
    held = [synth._build("held2a", [(128, 128, 4.0)], (0.8, 0.5), 0.0, seed=101),
            synth._build("held2b", [(64, 64, 12.0)], (0.8, 0.5), 0.0, seed=102)]
    need = 0.0
    for wl in held:
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        m, c, col, op = t(wl.mean), t(wl.chol), t(wl.color), t(wl.opacity)
        imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
        plan = G.RasterPlan(imgs, wl.n_gauss)
        plan.ensure_capacity(m, c)
        ws, exact = plan.new_workspace(dev), plan.new_output(dev)
        plan.forward(m, c, col, op, ws, exact)
        out = plan.new_output(dev)
        margin = 0.0
        while margin < 3.0:
            R = closed_form_radius(c, col, op, tau, margin)
            plan.forward(m, c, col, op, ws, out, R)
            if psnr(out, exact) >= target_db:
                break
            margin = round(margin + 0.05, 2)
        need = max(need, margin)
    return need


def pruned_comparison(G, synth, torch, np, names, reps):
    """Exact vs surrogate-pruned fwd+bwd on the wide-sigma DIV2K-sized
    workloads: train the radius network on labels the exact rasterizer
    measures on 10k seeded images, calibrate the closed-form control to
    >= 50 dB on held-out images, then time the three steps (each captured as
    one graph) and report the PSNR of each pruned render against the exact
    one."""
    from paper_2501_06838_amd.surrogate_train import train_radius_mlp
    tau = 4e-3
    log("surrogate: labels from the exact rasterizer on 10k images, training")
    net, info = train_radius_mlp(lambda k: synth.surrogate_training_batch(11, k), 600, 25, tau,
                                 steps=600, lr=3e-3, quantile=0.9, coverage=0.999)
    log(f"surrogate trained: margin {info['margin']:.3f}, loss {info['losses'][-1]:.4f}")
    cf_margin = calibrate_control(G, synth, torch, np, tau)
    log(f"closed-form control: margin {cf_margin} for >= 50.5 dB on held-out images")
    out = []
    for name in names:
        r = pruned_one(G, synth, torch, np, net, info, tau, cf_margin, name, reps)
        log(f"pruned ({name}): {r['pruned']['mp_s']} vs exact {r['exact']['mp_s']} MP/s "
            f"({r['speedup']}x) at {r['pruned']['psnr_db']} dB; control "
            f"{r['closed_form_control']['mp_s']} MP/s at {r['closed_form_control']['psnr_db']} dB")
        out.append(r)
    return out


def pruned_one(G, synth, torch, np, net, info, tau, cf_margin, name, reps):
    from paper_2501_06838_amd.surrogate import closed_form_radius, psnr
    B = Bench(G, synth, torch, np, name)
    dev = B.dev
    radius = torch.empty(B.n, device=dev)
    rcf = torch.empty(B.n, device=dev)
    results = {}
    exact_img = None
    for mode in ("exact", "pruned", "closed_form"):
        plan = G.RasterPlan(B.imgs, B.n)
        rad = None
        if mode == "pruned":
            net.radius_for(plan, B.chol, B.color, B.opacity, out=radius)
            rad = radius
        elif mode == "closed_form":
            closed_form_radius(B.chol, B.color, B.opacity, tau, cf_margin, out=rcf)
            rad = rcf
        plan.ensure_capacity(B.mean, B.chol, rad, headroom=1.05)
        ws, out, grads, loss = B.buffers(plan)

        def step():  # the radius is formed inside the step (one kernel)
            if mode == "pruned":
                net.radius_for(plan, B.chol, B.color, B.opacity, out=radius)
            elif mode == "closed_form":
                closed_form_radius(B.chol, B.color, B.opacity, tau, cf_margin, out=rcf)
            plan.step_l1(B.mean, B.chol, B.color, B.opacity, ws, out, B.target, grads,
                         radius=rad)

        step()
        torch.cuda.synchronize()
        npairs, overflow, _, nsup = plan.diagnostics(ws, support=True)
        if overflow:
            raise SystemExit("pair capacity overflow (pruned comparison)")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        warm_up(torch, g.replay, 5, 0.05)
        ms, brackets = time_graph(torch, g.replay, reps)
        r = {"ms_per_step": round(ms, 4), "brackets_ms": [round(x, 4) for x in brackets],
             "mp_s": round(plan.out_numel / 3 / (ms * 1e-3) / 1e6, 2),
             "tile_pairs": npairs, "support_pairs": nsup}
        if mode == "exact":
            exact_img = out.clone()
        else:
            r["psnr_db"] = round(psnr(out, exact_img), 2)
        if mode == "pruned":
            r["share_at_full_radius"] = round(float((radius >= 3.0).float().mean()), 4)
        results[mode] = r
        del g, ws, out, grads
    ex, pr, cf = results["exact"], results["pruned"], results["closed_form"]
    return {
        "workload": f"{name}: {WORKLOADS[name]}", "tau": tau, "exact": ex, "pruned": pr,
        "speedup": round(ex["ms_per_step"] / pr["ms_per_step"], 3),
        "closed_form_control": dict(cf, margin=cf_margin,
                                    calibration="smallest margin (0.05 grid) reaching 50.5 dB "
                                                "on held-out 128^2 x4 and 64^2 x12 images"),
        "speedup_vs_control": round(cf["ms_per_step"] / pr["ms_per_step"], 3),
        "control_speedup_vs_exact": round(ex["ms_per_step"] / cf["ms_per_step"], 3),
        "surrogate": {k: info[k] for k in ("train_rows", "calib_rows", "margin", "steps",
                                            "seconds_data", "seconds_train", "quantile",
                                            "coverage")},
        "launch": "each step (the pruned ones including their radius kernel) captured as one "
                  "HIP graph; median of three brackets",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config2a", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=0, help="0: autotuned launch configuration")
    ap.add_argument("--lds-batch", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pruned", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the other single workloads (config1, config2b)")
    ap.add_argument("--pruned-workload", default="config2a,config2b",
                    help="comma-separated, from config2a, config2b")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the r-window paper-shaped workloads and the head / PSNR kernels")
    ap.add_argument("--paper-scales", default="4,8",
                    help="comma-separated integer scales of the 720x720 r-window workload")
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="MIB",
                    help="finish with 5 plain device-to-device copies of MIB MiB (a known "
                         "byte count for scaling hardware traffic counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (--gpus 1): every workload here fits one "
              "MI355X; how a render would shard over several GPUs is described in the design "
              "notes, not measured.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2501_06838_amd as G
    import synth

    names = [n.strip() for n in args.pruned_workload.split(",") if n.strip()]
    for n in names:
        if n not in ("config2a", "config2b"):
            raise SystemExit(f"--pruned-workload: {n} is not config2a or config2b")
    torch.cuda.set_device(0)
    log("workload", args.workload)
    B = Bench(G, synth, torch, np, args.workload)
    if args.tile:
        launch = {"tile": args.tile, "lds_batch": args.lds_batch, "flags": 0}
        tuned = None
    else:
        launch, tuned, _ = autotune(B)
        log(f"autotuner picked {launch}")
    plan, _ = B.plan(launch)
    ws, out, grads, loss = B.buffers(plan)

    def step():
        plan.step_l1(B.mean, B.chol, B.color, B.opacity, ws, out, B.target, grads, loss=loss)

    step()
    torch.cuda.synchronize()
    npairs, overflow, n_invalid, n_support = plan.diagnostics(ws, support=True)
    if overflow:
        raise SystemExit("pair capacity overflow")
    log(f"tile pairs {npairs}, in-support pairs {n_support}, invalid {n_invalid}")
    graph = G.StepGraph(plan, B.mean, B.chol, B.color, B.opacity, ws, out, B.target, grads,
                        loss)
    # at least W warm-up replays, continued for 0.2 s of back-to-back work
    warm_up(torch, graph.launch, args.warmup, 0.2)

    # timed region: exactly K replays of the whole step
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    hr_px = plan.out_numel // 3
    value = hr_px / (ms_step * 1e-3) / 1e6
    if plan.diagnostics(ws)[1]:
        raise SystemExit("pair capacity overflow during replay")
    graph.close()

    # the dominant kernel's average duration: HIP events on its launch
    # stream around K back-to-back launches on the same binned batch (the
    # host's launch latency never empties the queue inside the bracket)
    fused_ms, fwd_ms, bwd_ms = tile_kernel_times(B, plan, ws, out, args.steps)
    step()  # leave the buffers as one eager step leaves them
    torch.cuda.synchronize()
    log(f"{ms_step:.4f} ms/step (graph replay); fused tile kernel {fused_ms * 1e3:.1f} us "
        f"(separate: fwd {fwd_ms * 1e3:.1f} us, bwd {bwd_ms * 1e3:.1f} us)")

    def tf(flopeq, ms):
        return n_support * flopeq / (ms * 1e-3) / 1e12
    fused_tflops = tf(FLOPEQ_FWD + FLOPEQ_BWD, fused_ms)
    roofline = {
        "bound": "alu", "kernel": "k_render_fused (forward + L1 gradient + backward per tile)",
        "achieved": round(fused_tflops, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
        "unit": "TFLOP/s", "frac": round(fused_tflops / PEAK_FP32_VECTOR_TFLOPS, 4),
        "traffic": traffic_bytes(args.workload, launch),
        "per_launch_flopeq": n_support * (FLOPEQ_FWD + FLOPEQ_BWD),
        "avg_launch_us": round(fused_ms * 1e3, 2),
        "fracs": roofline_fracs(n_support, hr_px, B.n, ms_step, fused_ms),
        "other": {name: {"achieved": round(tf(fe, ms), 3),
                         "frac": round(tf(fe, ms) / PEAK_FP32_VECTOR_TFLOPS, 4),
                         "avg_launch_us": round(ms * 1e3, 2)}
                  for name, fe, ms in (("k_render_fwd", FLOPEQ_FWD, fwd_ms),
                                       ("k_render_bwd (L1)", FLOPEQ_BWD, bwd_ms))},
    }

    # the same step with the other binning (counting with per-tile list sort,
    # or GS_FLAG_RADIX_SORT): same lists, bitwise; timed the same way
    radix = (launch["flags"] & G.GS_FLAG_RADIX_SORT) != 0
    other = "counting" if radix else "radix_sort"
    olaunch = dict(launch, flags=launch["flags"] ^ G.GS_FLAG_RADIX_SORT)
    binning = {"headline": "radix_sort" if radix else "counting",
               "ms_per_step": round(ms_step, 5),
               other: step_record(B, olaunch, args.steps, kernels=False)}
    log(f"{other} binning: {binning[other]['ms_per_step']:.4f} ms/step")
    del ws, out, grads

    # the vector-ALU probe: the FP32 rate the kernels can issue with packed
    # FP32 off, against which the fused kernel's rate is also given
    probe = valu_probe(torch)
    roofline["measured_fma_tflops"] = probe["fma_tflops"]
    roofline["frac_of_measured_fma"] = round(fused_tflops / probe["fma_tflops"], 4)
    log(f"valu probe: FMA {probe['fma_tflops']} TFLOP/s, exp2 {probe['exp2_per_s']:.3g}/s, "
        f"mask step cycles {probe['mask_step_cycles']}")

    others = None
    if not args.no_others:
        others = []
        for name in ("config1", "config2b", "config2a"):
            if name == args.workload:
                continue
            log("workload", name)
            others.append(step_record(Bench(G, synth, torch, np, name),
                                      {"tile": 16, "lds_batch": 96, "flags": 0}, args.steps))
    pruned = None
    if not args.no_pruned:
        pruned = pruned_comparison(G, synth, torch, np, names, args.steps)
    batched = None
    if not args.no_batched:
        batched = batched_uneven(G, synth, torch, np, max(20, args.steps))
        d = batched["default_launch"]
        d = batched[d["same_as"]] if "same_as" in d else d
        log(f"batched: default launch {d['mp_s']} MP/s")
    paper = extras = None
    if not args.no_paper:
        paper = paper_window(G, synth, torch, np,
                             [int(x) for x in args.paper_scales.split(",") if x.strip()],
                             args.steps)
        extras = head_and_psnr(G, synth, torch, np, max(20, args.steps))
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(B.wl, args.cpu_seconds)
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "HR megapixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "path": "exact 3-sigma support", "launch_config": launch,
                   "autotune_ms": tuned, "hr_pixels": hr_px, "gaussians": B.n,
                   "tile_pairs": npairs, "support_pairs": n_support,
                   "launch": "whole step captured in one HIP graph, replayed"},
        "roofline": roofline, "valu_probe": probe, "cpu_baseline": cpu,
        "surrogate_pruned": pruned,
        "workloads": others, "batched_uneven": batched, "binning": binning,
        "paper_window": paper, "head_psnr": extras,
    }
    print(json.dumps(rec), flush=True)
    if args.calibration_copy > 0:
        n = args.calibration_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=B.dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 5 x {args.calibration_copy} MiB")


if __name__ == "__main__":
    main()
