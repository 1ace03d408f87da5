#!/usr/bin/env python
"""Newton sweeps/s of the stochastic local-Newton 3DGS step on one MI355X.

Workload: 1M Gaussians (SH degree 3) on 20 random spheres/planes, 150 cameras
on a radius-4 Fibonacci sphere, primary target 1920x1080 plus its 3 nearest
cameras as half-resolution secondary targets (Sec. 4.1-4.3).  One step is one
full sweep: render + accumulate the primary and the three secondaries, solve
every kernel's local Newton systems and apply them.  Targets are rendered from
the seeded ground truth and are resident in HBM before timing starts; the
state being trained is a perturbed copy of the ground truth (synthetic data,
standing in for the paper's photographic datasets).

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton sweeps/s, 1M Gaussians @1080p: plain FP32 vs mixed+learned at equal PSNR"

# Peak figures of one MI355X (published): HBM3E bandwidth and the FP32 vector rate.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3

# Algorithmic FLOPs per unit of work, counted from the kernel sources:
#   forward: per (pixel, list entry) evaluation of the splat (offset, frame rotation,
#            quadratic form, exp, alpha, threshold tests) and per contribution the blend.
#   backward: the same evaluation, and per contributing (pixel, splat) pair the
#            44 projected-space gradient/Hessian terms.
FLOP_EVAL = 18
FLOP_FWD_BLEND = 9
FLOP_BWD_TERMS = 156


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def gpu_run(args):
    import numpy as np
    import torch

    from paper_2501_13975_amd import gsn
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    from synth.scenes import make_config, view_order

    t0 = time.time()
    cfg = make_config(args.config)
    dev = torch.device("cuda", 0)
    log(f"[bench] generated {args.config}: {cfg.n} kernels, {len(cfg.cams)} cameras ({time.time() - t0:.1f}s)")
    # targets: the ground truth rendered by the library, resident on the device
    gt = gsn.DeviceGaussians.from_host(cfg.gt, dev)
    ctx = gsn.Context(dev)
    fr = ctx.frame()
    ro = gsn.render_opts()
    targets = []
    for c in cfg.cams:
        img = torch.empty(3, c.height, c.width, dtype=torch.float32, device=dev)
        ctx.render(gt, gsn.camera(c), ro, fr, img)
        targets.append(img)
    torch.cuda.synchronize(dev)
    fr.close()
    ctx.close()
    del gt
    log(f"[bench] rendered {len(targets)} targets ({time.time() - t0:.1f}s)")
    g = gsn.DeviceGaussians.from_host(cfg.init, dev)
    tr = LocalNewtonTrainer(g, cfg.cams, targets, n_secondary=cfg.n_secondary)
    order = np.concatenate([view_order(len(cfg.cams), e) for e in range(4)])
    for i in range(args.warmup):
        tr.sweep(int(order[i]))
    torch.cuda.synchronize(dev)
    log(f"[bench] warmup {args.warmup} sweeps done ({time.time() - t0:.1f}s)")
    tr.ctx.profile_enable(True)
    torch.cuda.synchronize(dev)
    start = time.perf_counter()
    for i in range(args.steps):
        tr.sweep(int(order[args.warmup + i]))
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - start
    stages, counts = tr.ctx.profile_read()
    tr.ctx.profile_enable(False)
    loss = tr.loss.cpu().numpy()
    log(f"[bench] timed {args.steps} sweeps in {elapsed:.3f}s; stage ms: "
        + ", ".join(f"{k}={v[0]:.1f}" for k, v in stages.items()))
    tr.close()
    return elapsed, stages, counts, loss, cfg


def roofline(stages, counts, steps):
    """Roofline figure of the stage that takes the most time."""
    dom = max(stages, key=lambda s: stages[s][0])
    ms, launches = stages[dom]
    per_launch_s = ms * 1e-3 / max(launches, 1)
    if dom == "raster_bwd":
        flops = FLOP_EVAL * counts["bwd_evals"] + FLOP_BWD_TERMS * counts["bwd_active"]
        achieved = flops / max(launches, 1) / per_launch_s / 1e12
        return dict(kernel="raster_bwd", bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP32_TFLOPS, 5), traffic=None,
                    avg_launch_ms=round(ms / max(launches, 1), 4), launches=launches)
    if dom == "raster_fwd":
        flops = FLOP_EVAL * counts["fwd_evals"] + FLOP_FWD_BLEND * counts["bwd_active"]
        achieved = flops / max(launches, 1) / per_launch_s / 1e12
        return dict(kernel="raster_fwd", bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS,
                    unit="TFLOP/s", frac=round(achieved / PEAK_FP32_TFLOPS, 5), traffic=None,
                    avg_launch_ms=round(ms / max(launches, 1), 4), launches=launches)
    # sort/bin: 28 algorithmic bytes per (tile, kernel) pair (write key/value, read per tile, write list)
    nbytes = 28.0 * counts["pairs"]
    achieved = nbytes / max(launches, 1) / per_launch_s / 1e9
    return dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                frac=round(achieved / PEAK_HBM_GBS, 5), traffic=None, avg_launch_ms=round(ms / max(launches, 1), 4),
                launches=launches)


def cpu_baseline(cfg, budget_s):
    """The FP64 oracle on a bounded sample of the same sweep, scaled to sweeps/s."""
    import numpy as np

    from oracle import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = O.opts(npix_primary=cfg.cams[0].width * cfg.cams[0].height)
    cam = cfg.cams[0]
    t = time.perf_counter()
    target = O.render(cfg.gt, cam, o).img
    fr = O.render(cfg.init, cam, o)
    t_render = time.perf_counter() - t
    # loss maps on a 256x256 crop, scaled by pixel count
    y0, x0 = cam.height // 2 - 128, cam.width // 2 - 128
    crop = (slice(None), slice(y0, y0 + 256), slice(x0, x0 + 256))
    t = time.perf_counter()
    _, dL, hd = O.loss(fr.img[crop], target[crop], 0.2)
    t_loss = (time.perf_counter() - t) * (cam.width * cam.height) / (256 * 256)
    dL_full = np.zeros_like(fr.img)
    hd_full = np.zeros_like(fr.img)
    dL_full[crop], hd_full[crop] = dL, hd
    # per-kernel blocks for random visible kernels until the budget is spent (the cost of a
    # kernel's blocks does not depend on the values of the loss maps)
    vis = np.nonzero(fr.vis)[0]
    rng = np.random.default_rng(0)
    sel = rng.permutation(vis)
    done, t_blocks, batch = 0, 0.0, 8
    spent = t_render + t_loss * (256 * 256) / (cam.width * cam.height)
    while done < len(sel) and spent + t_blocks < budget_s:
        t = time.perf_counter()
        O.blocks(cfg.init, fr, dL_full, hd_full, sel[done:done + batch])
        t_blocks += time.perf_counter() - t
        done += batch
    t_blocks_all = t_blocks * len(vis) / max(done, 1)
    # secondaries: three views at a quarter of the pixels each
    sweep_s = (t_render + t_loss + t_blocks_all) * (1.0 + 3 * 0.25)
    return dict(value=round(1.0 / sweep_s, 6), unit="sweeps/s", cores=threads, kind="oracle",
                sample=(f"FP64 oracle on the primary 1920x1080 view of the same workload: full render "
                        f"({t_render:.1f}s), loss maps on a 256x256 crop scaled by pixel count, per-kernel "
                        f"blocks for {done} of {len(vis)} visible kernels scaled by count; three half-resolution "
                        f"secondaries counted as 0.25 of the primary each"))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs the training step on a single MI355X "
              "(how it would shard across GPUs is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    elapsed, stages, counts, loss, cfg = gpu_run(args)
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.steps / elapsed
    rl = roofline(stages, counts, args.steps)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on a bounded sample ...")
        cpu = cpu_baseline(cfg, args.cpu_budget)
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "sweeps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{cfg.n} Gaussians SH3 on random spheres/planes, {len(cfg.cams)} cameras, "
                                f"primary {cfg.width}x{cfg.height} + {cfg.n_secondary} KNN secondaries at "
                                f"{cfg.width // 2}x{cfg.height // 2}; plain FP32 form"),
                   "gaussians": cfg.n, "width": cfg.width, "height": cfg.height, "cameras": len(cfg.cams),
                   "secondaries": cfg.n_secondary, "form": "plain"},
        "gaussians_updated_per_s": round(value * cfg.n, 1),
        "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
        "counts_per_step": {k: int(v / args.steps) for k, v in counts.items()},
        "roofline": rl,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
