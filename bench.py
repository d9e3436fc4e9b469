"""Throughput of the scale-aware 2D Gaussian rasterizer on one MI355X.

One step = one forward + L1-loss gradient + backward of the whole hot path
(support boxes, tile binning, radix sort, tile ranges, tile render, loss
gradient, tile backward render, per-Gaussian gradients) over the workload's
batch, every kernel from the HIP library.  Inputs are resident in HBM before
timing starts.

Default workload: 16 images of 64x64 LR, 4,096 Gaussians each, rendered at
s = 3.7 to 237x237 (seeded synthetic Gaussians, uniform random target).

    python bench.py [--steps K] [--warmup W] [--workload config1]

Prints ONE JSON line (see the metric, roofline and cpu_baseline keys).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
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

# HBM traffic of one fused tile-kernel launch (k_render_fused) on config1 at
# tile 16, LDS batch 96, from two rocprofv3 --pmc passes (FETCH_SIZE,
# WRITE_SIZE; KiB per dispatch, averaged over the dispatches), each scaled by
# what the same counter reads for a plain 256 MiB device copy: FETCH_SIZE
# reads 131,084.6 KiB (factor 2.0), WRITE_SIZE 262,144 KiB (factor 1.0).  Valid
# only while the render sources hash to `sources`; otherwise null.
# The same profile's VALU counters: busy = SQ_ACTIVE_INST_VALU x 4 / 1,024
# SIMDs / (GRBM_GUI_ACTIVE / 8 XCDs), per dispatch.
TRAFFIC = {"workload": "config1", "launch": {"tile": 16, "lds_batch": 96, "flags": 0},
           "sources": "3b348b0d821e0322",
           "fetch_kib": 11269.8, "write_kib": 17600.0, "fetch_factor": 2.0, "write_factor": 1.0,
           "sq_active_inst_valu": 22810120, "grbm_gui_active": 1133433}
TRAFFIC_SOURCES = ("paper_2501_06838_amd/csrc/gs_render.hip", "paper_2501_06838_amd/csrc/gs_internal.h")


def render_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_valid(workload, launch):
    T = TRAFFIC
    return (workload == T["workload"] and launch == T["launch"]
            and render_sources_hash() == T["sources"])


def traffic_bytes(workload, launch):
    T = TRAFFIC
    if not profile_valid(workload, launch):
        return None
    return round(T["fetch_kib"] * 1024 * T["fetch_factor"] + T["write_kib"] * 1024 * T["write_factor"])


def valu_busy(workload, launch):
    """Fraction of the SIMDs' cycles issuing VALU work in the profiled fused
    kernel (profiles/config1_k_render_fused_valu.md), or None."""
    T = TRAFFIC
    if not profile_valid(workload, launch):
        return None
    return round(T["sq_active_inst_valu"] * 4 / 1024 / (T["grbm_gui_active"] / 8), 3)


WORKLOADS = {
    "config1": "16 x 64x64 LR (4,096 Gaussians each) -> 237x237 at s=3.7, fwd+bwd, L1 loss",
    "config0": "48x48 LR (2,304 Gaussians) -> 192x192 at s=4, fwd+bwd, L1 loss",
    "config2a": "512x512 LR (262,144 Gaussians) -> 2048x2048 at s=4, fwd+bwd, L1 loss",
    "config2b": "256x256 LR (65,536 Gaussians) -> 3072x3072 at s=12, fwd+bwd, L1 loss",
    "config3": "64 uneven images, LR U{48..256}^2 +25% Gaussians, s~U[1.5,12], fwd+bwd, L1 loss",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(wl, seconds: float):
    """The FP64 C oracle (single thread) on whole images of the same workload,
    round-robin until `seconds` have elapsed: forward, L1 gradient, backward."""
    import numpy as np
    from oracle import oracle as O
    O.lib()
    t0 = time.perf_counter()
    px = 0
    n = 0
    k = 0
    while True:
        im = wl.images[k % len(wl.images)]
        sl = wl.image_slice(k % len(wl.images))
        img = O.forward(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl], wl.color[sl],
                        wl.opacity[sl])
        tgt = wl.target[k % len(wl.images)]
        g = np.sign(img - tgt) / img.size
        O.backward(im.lr_h, im.lr_w, im.scale, wl.mean[sl], wl.chol[sl], wl.color[sl],
                   wl.opacity[sl], g)
        px += img.shape[1] * img.shape[2]
        n += 1
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {
        "value": px / el / 1e6, "unit": "HR megapixels/s", "cores": 1, "kind": "oracle",
        "sample": f"{n} whole images of the workload ({px} HR px) in {el:.1f} s: FP64 C "
                  f"oracle, one thread, forward + L1 gradient + backward",
        "cpu": platform.processor() or platform.machine(), "host_cpus": os.cpu_count(),
    }


def batched_uneven(args, G, synth, torch, np):
    """The serving-style batch: 64 uneven images rendered fwd+bwd in one
    captured step, with the launch configuration (tile, LDS batch,
    persistent longest-first kernels) picked by the autotuner; the default
    launch (tile 16, one workgroup per tile) is timed beside it."""
    from paper_2501_06838_amd.autotune import tune
    dev = torch.device("cuda:0")
    log("batched: config3 (64 uneven images)")
    wl = synth.config3(with_target=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mean, chol, color, opacity = t(wl.mean), t(wl.chol), t(wl.color), t(wl.opacity)
    imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
    plan0 = G.RasterPlan(imgs, wl.n_gauss, tile=16)
    target = plan0.pack([t(x) for x in wl.target])
    wl.target = None
    t0 = time.perf_counter()
    res = tune(imgs, mean, chol, color, opacity, target, reps=5, warmup=2)
    t_tune = time.perf_counter() - t0
    best = res["config"]
    log(f"batched: autotuner picked {best} in {t_tune:.1f} s")
    hr_px = plan0.out_numel // 3
    out = {"workload": "config3: " + WORKLOADS["config3"], "images": len(imgs),
           "hr_pixels": hr_px, "gaussians": int(mean.shape[0]),
           "autotune": {"config": best, "seconds": round(t_tune, 2),
                        "timings_ms": [[c["config"]["tile"], c["config"]["lds_batch"],
                                        c["config"]["flags"], c["ms"]] for c in res["timings"]]}}
    for name, cfg in (("tuned", best), ("default_launch", {"tile": 16, "lds_batch": 0,
                                                           "flags": 0})):
        plan = G.RasterPlan(imgs, int(mean.shape[0]), **cfg)
        pairs = plan.ensure_capacity(mean, chol)
        ws, img = plan.new_workspace(dev), plan.new_output(dev)
        n = int(mean.shape[0])
        grads = (torch.empty(n, 2, device=dev), torch.empty(n, 3, device=dev),
                 torch.empty(n, 3, device=dev), torch.empty(n, device=dev))
        loss = torch.zeros((), dtype=torch.float64, device=dev)
        graph = G.StepGraph(plan, mean, chol, color, opacity, ws, img, target, grads, loss)
        for _ in range(3):
            graph.launch()
        torch.cuda.synchronize()
        steps = max(5, args.steps // 5)
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.launch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if plan.diagnostics(ws)[1]:
            raise SystemExit("pair capacity overflow (batched)")
        graph.close()
        out[name] = {"ms_per_step": round(ms, 4), "mp_s": round(hr_px / (ms * 1e-3) / 1e6, 2),
                     "tile_pairs": pairs, "steps": steps, "config": cfg}
        del ws, img, grads
    out["launch"] = "each step captured as one HIP graph, replayed"
    return out


def pruned_comparison(args, G, synth, torch, np):
    """Exact vs surrogate-pruned fwd+bwd on a wide-sigma DIV2K-sized workload:
    train the radius network on labels the exact rasterizer measures on 10k
    seeded images, then time both steps (each captured as one graph) and
    report the PSNR of the pruned render against the exact one."""
    from paper_2501_06838_amd.surrogate_train import train_radius_mlp
    tau = 4e-3
    log("surrogate: labels from the exact rasterizer on 10k images, training")
    net, info = train_radius_mlp(lambda k: synth.surrogate_training_batch(11, k), 600, 25, tau,
                                 steps=600, lr=3e-3, quantile=0.9, coverage=0.999)
    log(f"surrogate trained: margin {info['margin']:.3f}, loss {info['losses'][-1]:.4f}")
    out_list = []
    names = [n.strip() for n in args.pruned_workload.split(",") if n.strip()]
    for name in names:
        if name not in ("config2a", "config2b"):
            raise SystemExit(f"--pruned-workload: {name} is not config2a or config2b")
    for name in names:
        r = pruned_one(args, G, synth, torch, np, net, info, tau, name)
        log(f"pruned ({name}): {r['pruned']['mp_s']} vs exact {r['exact']['mp_s']} MP/s "
            f"({r['speedup']}x) at {r['pruned']['psnr_db']} dB")
        out_list.append(r)
    return out_list


def pruned_one(args, G, synth, torch, np, net, info, tau, name):
    """One workload of the pruned comparison with the trained network."""
    from paper_2501_06838_amd.surrogate import psnr
    dev = torch.device("cuda:0")
    wl = synth.by_name(name, with_target=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mean, chol, color, opacity = t(wl.mean), t(wl.chol), t(wl.color), t(wl.opacity)
    imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
    target = None
    results = {}
    radius = torch.empty(wl.n_gauss, device=dev)
    # closed-form control radius sqrt(2 ln(alpha max(c) K / tau)), K = 1/(2 pi l11 l22)
    K = 1.0 / (2 * np.pi * np.float64(wl.chol[:, 0]) * np.float64(wl.chol[:, 2]))
    arg = np.float64(wl.opacity) * np.float64(wl.color).max(1) * K / tau
    rcf = t(np.minimum(np.sqrt(2 * np.log(np.maximum(arg, 1.0))), 3.0).astype(np.float32))
    for mode in ("exact", "pruned", "closed_form"):
        plan = G.RasterPlan(imgs, wl.n_gauss, tile=args.tile or 16)
        if target is None:
            target = plan.pack([t(x) for x in wl.target])
        rad = None
        if mode == "pruned":
            net.radius_for(plan, chol, color, opacity, out=radius)
            rad = radius
        elif mode == "closed_form":
            rad = rcf
        plan.ensure_capacity(mean, chol, rad, headroom=1.05)
        ws, out = plan.new_workspace(dev), plan.new_output(dev)
        grads = (torch.empty(wl.n_gauss, 2, device=dev), torch.empty(wl.n_gauss, 3, device=dev),
                 torch.empty(wl.n_gauss, 3, device=dev), torch.empty(wl.n_gauss, device=dev))

        def step():
            if mode == "pruned":  # the radius is predicted inside the step (one kernel)
                net.radius_for(plan, chol, color, opacity, out=radius)
            plan.step_l1(mean, chol, color, opacity, ws, out, target, grads, radius=rad)

        step()
        torch.cuda.synchronize()
        npairs, overflow, _, nsup = plan.diagnostics(ws, support=True)
        if overflow:
            raise SystemExit("pair capacity overflow (pruned comparison)")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step()
        for _ in range(10):
            g.replay()
        torch.cuda.synchronize()
        n = max(50, args.steps)
        t0 = time.perf_counter()
        for _ in range(n):
            g.replay()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / n
        results[mode] = {"ms_per_step": round(ms, 4),
                         "mp_s": round(plan.out_numel / 3 / (ms * 1e-3) / 1e6, 2),
                         "tile_pairs": npairs, "support_pairs": nsup, "image": out.clone()}
        if mode != "exact":
            results[mode]["psnr_db"] = round(psnr(out, results["exact"]["image"]), 2)
        if mode == "pruned":
            results[mode]["share_at_full_radius"] = round(float((radius >= 3.0).float().mean()), 4)
        del g
    for r in results.values():
        r.pop("image")
    return {
        "workload": f"{name}: {WORKLOADS[name]}",
        "tau": tau, "exact": results["exact"], "pruned": results["pruned"],
        "speedup": round(results["exact"]["ms_per_step"] / results["pruned"]["ms_per_step"], 3),
        "closed_form_control": results["closed_form"],
        "surrogate": {k: info[k] for k in ("train_rows", "calib_rows", "margin", "steps",
                                            "seconds_data", "seconds_train", "quantile",
                                            "coverage")},
        "launch": "each step (the pruned one including feature + MLP radius kernels) "
                  "captured as one HIP graph",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="config1", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=0, help="0: autotuned launch configuration")
    ap.add_argument("--lds-batch", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pruned", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--pruned-workload", default="config2a,config2b",
                    help="comma-separated, from config2a, config2b")
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="MIB",
                    help="finish with 5 plain device-to-device copies of MIB MiB (a known "
                         "byte count for scaling hardware traffic counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (--gpus 1): the library renders a batch on "
              "a single MI355X; sharding over several GPUs is described, not measured.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2501_06838_amd as G
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("workload", args.workload)
    wl = synth.by_name(args.workload, with_target=True)
    if wl.target is None:
        raise SystemExit("workload has no target")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mean, chol, color, opacity = t(wl.mean), t(wl.chol), t(wl.color), t(wl.opacity)
    imgs = [(im.lr_h, im.lr_w, im.scale, im.g_begin, im.g_count) for im in wl.images]
    target = G.RasterPlan(imgs, wl.n_gauss).pack([t(x) for x in wl.target])
    if args.tile:
        launch = {"tile": args.tile, "lds_batch": args.lds_batch, "flags": 0}
        tuned = None
    else:
        from paper_2501_06838_amd.autotune import tune
        res = tune(imgs, mean, chol, color, opacity, target, reps=5, warmup=2)
        launch = res["config"]
        tuned = [[c["config"]["tile"], c["config"]["lds_batch"], c["config"]["flags"], c["ms"]]
                 for c in res["timings"]]
        log(f"autotuner picked {launch}")
    plan = G.RasterPlan(imgs, wl.n_gauss, **launch)
    plan.ensure_capacity(mean, chol)
    ws = plan.new_workspace(dev)
    out = plan.new_output(dev)
    loss_acc = torch.zeros((), dtype=torch.float64, device=dev)
    grads = (torch.empty(wl.n_gauss, 2, device=dev), torch.empty(wl.n_gauss, 3, device=dev),
             torch.empty(wl.n_gauss, 3, device=dev), torch.empty(wl.n_gauss, device=dev))
    stream = torch.cuda.current_stream()

    def step():
        # binning, fused tile kernel (render + L1 gradient + backward), gradients, loss
        plan.step_l1(mean, chol, color, opacity, ws, out, target, grads, loss=loss_acc)

    # one eager step, then the step captured as one HIP graph
    step()
    torch.cuda.synchronize()
    npairs, overflow, n_invalid, n_support = plan.diagnostics(ws, support=True)
    if overflow:
        raise SystemExit("pair capacity overflow")
    log(f"tile pairs {npairs}, in-support pairs {n_support}, invalid {n_invalid}")
    graph = G.StepGraph(plan, mean, chol, color, opacity, ws, out, target, grads, loss_acc)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()

    # timed region: K replays of the whole step
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    hr_px = plan.out_numel // 3
    value = hr_px / (ms_step * 1e-3) / 1e6
    if plan.diagnostics(ws)[1]:
        raise SystemExit("pair capacity overflow during replay")

    # per-kernel durations: HIP events on the launch stream around K
    # back-to-back launches of the single-kernel entry points on the bound
    # batch (same inputs, same launch config), so the host's launch latency
    # never leaves the queue empty inside the bracket.  The step's tile kernel
    # is the fused one; the separate forward and backward tile kernels are
    # timed too, for reference.
    def bracket(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        return a, b
    plan.bin(mean, chol, color, opacity, ws)
    plan.render_fused_l1(ws, out, target)
    ev_fused = bracket(lambda: plan.render_fused_l1(ws, out, target))
    ev_fwd = bracket(lambda: plan.render(ws, out))
    ev_bwd = bracket(lambda: plan.render_backward_l1(ws, out, target))
    torch.cuda.synchronize()
    fused_ms, fwd_ms, bwd_ms = (a.elapsed_time(b) / args.steps for a, b in (ev_fused, ev_fwd, ev_bwd))
    # leave the buffers as one eager step leaves them
    step()
    torch.cuda.synchronize()
    log(f"{ms_step:.4f} ms/step (graph replay); fused tile kernel {fused_ms * 1e3:.1f} us "
        f"(separate: fwd {fwd_ms * 1e3:.1f} us, bwd {bwd_ms * 1e3:.1f} us)")
    graph.close()

    def tf(flopeq, ms):
        return n_support * flopeq / (ms * 1e-3) / 1e12
    fused_tflops = tf(FLOPEQ_FWD + FLOPEQ_BWD, fused_ms)
    roofline = {
        "bound": "alu", "kernel": "k_render_fused (forward + L1 gradient + backward per tile)",
        "achieved": round(fused_tflops, 3),
        "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
        "frac": round(fused_tflops / PEAK_FP32_VECTOR_TFLOPS, 4),
        "traffic": traffic_bytes(args.workload, launch),
        "valu_busy": valu_busy(args.workload, launch),
        "per_launch_flopeq": n_support * (FLOPEQ_FWD + FLOPEQ_BWD),
        "avg_launch_us": round(fused_ms * 1e3, 2),
        "other": {name: {"achieved": round(tf(fe, ms), 3),
                         "frac": round(tf(fe, ms) / PEAK_FP32_VECTOR_TFLOPS, 4),
                         "avg_launch_us": round(ms * 1e3, 2)}
                  for name, fe, ms in (("k_render_fwd", FLOPEQ_FWD, fwd_ms),
                                       ("k_render_bwd (L1)", FLOPEQ_BWD, bwd_ms))},
    }
    # the same step with the radix-sort binning (GS_FLAG_RADIX_SORT): same
    # lists, bitwise; timed the same way
    rplan = G.RasterPlan(imgs, wl.n_gauss, tile=launch["tile"], lds_batch=launch["lds_batch"],
                         flags=launch["flags"] | G.GS_FLAG_RADIX_SORT)
    rplan.ensure_capacity(mean, chol)
    rws = rplan.new_workspace(dev)
    rgraph = G.StepGraph(rplan, mean, chol, color, opacity, rws, out, target, grads, loss_acc)
    for _ in range(args.warmup):
        rgraph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rgraph.launch()
    torch.cuda.synchronize()
    radix_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    rgraph.close()
    del rws
    binning = {"default": "pairs counted into their tiles, each tile's list sorted",
               "ms_per_step": round(ms_step, 5), "radix_sort_ms_per_step": round(radix_ms, 5)}
    log(f"radix-sort binning: {radix_ms:.4f} ms/step (counting: {ms_step:.4f})")
    pruned = None
    if not args.no_pruned:
        pruned = pruned_comparison(args, G, synth, torch, np)
    batched = None
    if not args.no_batched:
        batched = batched_uneven(args, G, synth, torch, np)
        log(f"batched: tuned {batched['tuned']['mp_s']} MP/s, default launch "
            f"{batched['default_launch']['mp_s']} MP/s")
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(wl, args.cpu_seconds)
    rec = {
        "metric": METRIC, "value": round(value, 3), "unit": "HR megapixels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "path": "exact 3-sigma support", "launch_config": launch,
                   "autotune_ms": tuned,
                   "hr_pixels": hr_px, "gaussians": wl.n_gauss, "tile_pairs": npairs,
                   "support_pairs": n_support,
                   "launch": "whole step captured in one HIP graph, replayed"},
        "roofline": roofline, "cpu_baseline": cpu, "surrogate_pruned": pruned,
        "batched_uneven": batched, "binning": binning,
    }
    print(json.dumps(rec), flush=True)
    if args.calibration_copy > 0:
        n = args.calibration_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: 5 x {args.calibration_copy} MiB")


if __name__ == "__main__":
    main()
