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

# Peak figures of one MI355X.  HBM3E: 8 TB/s (published).  Vector ALU: the published FP32 vector
# peak 157.3 TFLOP/s (packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2 FLOP per FMA x 2.4 GHz).
# The unpacked rate, 78.6 TFLOP/s (also the FP64 vector peak), is reported beside it: this library
# is built without packed FP32 instructions, so that is the rate its FP32 code can reach.
PEAK_HBM_GBS = 8000.0
# every kernel's steps times its overlap share (gsn_solve_opts.overlap_scale; --no-overlap turns it off)
OVERLAP = 1
PEAK_ALU_TFLOPS = 157.3
PEAK_ALU_UNPACKED_TFLOPS = 78.6

# Algorithmic FLOPs per unit of work, counted from the kernel sources:
#   one (pixel, list entry) evaluation of a splat: offset with the mean's low word (4),
#     rotation into the principal frame (6), quadratic form and exponent scale (6), exp (1),
#     times opacity (1) = 18;
#   one forward contribution: transmittance update (2), alpha T (1), three double
#     colour accumulations (6) = 9;
#   one backward contributing (pixel, splat) pair: its evaluation (18), transmittance and
#     colour-behind bookkeeping with the alpha derivatives a_ch (35), offsets in the principal
#     frame (10), the 44 projected-space terms (115) and their accumulation (44) = 222.
# The backward pass evaluates a (pixel, entry) again only past the batches whose composited
# entries the forward pass recorded (counted as bwd_evals, 18 each).
FLOP_EVAL = 18
FLOP_FWD_BLEND = 9
FLOP_BWD_PAIR = 222
# Algorithmic bytes per unit (the method's own traffic, not this implementation's):
#   a consumed list entry (staged before its tile finished), forward or backward: its index (4) and
#     the projected record it reads (36) = 40;
#   per pixel: the forward pass writes colour, transmittance and stopping index (20), the loss maps
#     are written and read (48: dL and h, 3 channels each), the backward pass reads maps, colour and
#     stopping index (44);
#   per kernel and view: the 43 projected-space statistics written and read once (172);
#   per emitted (tile, kernel) pair: key/value write, per-tile bucket read, list write (28).
BYTES_ENTRY = 40
BYTES_FWD_PIXEL = 20
BYTES_BWD_PIXEL = 44
BYTES_ZSTATS = 172
BYTES_PAIR = 28


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _targets(cfg, dev):
    """Ground-truth renders by the library, resident on the device."""
    import torch

    from paper_2501_13975_amd import gsn
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
    return targets


def _trainer(cfg, targets, dev, learned_every=0, step_frac=1.0, n_secondary=None, gauss_newton=False,
             reserve=False, precision=None):
    """The plain form (FP64 small solves), or with learned_every the mixed + learned form (BF16
    matrix-core colour Grams, FP32 solves with FP64 for flagged systems, single-precision render and
    accumulation, learned step scale); precision=1 without learned_every is the mixed form alone.
    n_secondary overrides the workload's |N_t|; gauss_newton selects the local Gauss-Newton blocks;
    reserve sizes every frame once, so that sweeps never wait for the device."""
    from paper_2501_13975_amd import gsn
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    from synth.mlp_init import init_params
    g = gsn.DeviceGaussians.from_host(cfg.init, dev)
    prec = (1 if learned_every else 0) if precision is None else precision
    kw = {"step_frac": step_frac, "precision": prec, "overlap": OVERLAP}
    K = cfg.n_secondary if n_secondary is None else n_secondary
    tr = LocalNewtonTrainer(g, cfg.cams, targets, n_secondary=K, solve_kw=kw, gauss_newton=gauss_newton)
    if learned_every:
        tr.enable_learned(init_params(0), every=learned_every, lr=1e-2)
    if reserve:
        tr.reserve_frames()
    return tr


def _sweep(tr, t, i, learned, mask=31):
    if learned:
        tr.sweep_learned(t, i, mask)
    else:
        tr.sweep(t, mask)


def _timed(tr, order, warmup, steps, learned, dev, profile=True, wave_steps=False):
    """Times `steps` sweeps after `warmup` untimed ones (the host clock around a synchronised
    loop).  With profile, the library also times every stage with HIP events and counts its work
    (a few microseconds per stage): the stage times and counters are returned."""
    import torch
    for i in range(warmup):
        _sweep(tr, int(order[i]), i, learned)
    torch.cuda.synchronize(dev)
    if profile:
        tr.ctx.profile_enable(True, steps=wave_steps)
    torch.cuda.synchronize(dev)
    start = time.perf_counter()
    for i in range(steps):
        _sweep(tr, int(order[warmup + i]), warmup + i, learned)
    torch.cuda.synchronize(dev)
    elapsed = time.perf_counter() - start
    stages, counts = None, None
    if profile:
        stages, counts = tr.ctx.profile_read()
        tr.ctx.profile_enable(False)
    return elapsed, stages, counts


def _rate_and_profile(tr, order, warmup, steps, learned, dev):
    """Seconds for `steps` unprofiled sweeps after `warmup`, then the stage times and counters of
    `steps` more sweeps run with the library's profiler on."""
    el, _, _ = _timed(tr, order, warmup, steps, learned, dev, profile=False)
    _, st, cn = _timed(tr, order[warmup + steps:], 0, steps, learned, dev)
    return el, st, cn


def _mixed_vs_plain(cfg, targets, dev, t, step_frac):
    """One sweep's blocks and steps of the mixed form against the plain form's on the same state
    (training image t): per group the largest difference relative to the plain form's largest
    entry, over the kernels the primary sees; steps over the kernels whose five decisions agree
    (largest, median, 99th and 99.9th percentile over the kernels), and the share of solved kernels
    whose decisions differ.  The plain form matches the FP64
    oracle to about 1e-6 (the parity tests), so these are the mixed form's errors to that accuracy."""
    import torch
    from paper_2501_13975_amd import gsn
    res = {}
    trs = [_trainer(cfg, targets, dev, 0, step_frac, precision=p) for p in (0, 1)]
    blocks, steps, flags = [], [], []
    for tr in trs:
        tr.accumulate(t)
        tr.ctx.local_newton_solve(tr.g, tr.ccams[t], tr.blocks, tr.solve_opts(t), tr.steps)
        st, fl = tr.steps.view()
        blocks.append(tr.blocks.view().clone())
        steps.append(st.clone())
        flags.append(fl.clone())
    for tr in trs:
        tr.close()
    torch.cuda.synchronize(dev)
    seen = blocks[0][29] > 0
    V = trs[0].blocks.n_views
    colour = [gsn.GSN_BLK_BASE + gsn.GSN_BLK_VIEW * v + r for v in range(V) for r in range(6)]

    def rel(a, b, rows, cols, quantiles=False):
        x, y = a[rows][:, cols].double(), b[rows][:, cols].double()
        den = float(y.abs().max()) if y.numel() else 0.0
        if den <= 0:
            return 0.0
        d = (x - y).abs().amax(0) / den  # per kernel: its largest difference in the group
        if not quantiles:
            return round(float(d.max()), 8)
        q = torch.quantile(d, torch.tensor([0.5, 0.99, 0.999], dtype=d.dtype, device=d.device)).tolist()
        return {"max": round(float(d.max()), 8), "p50": round(q[0], 10), "p99": round(q[1], 8), "p999": round(q[2], 8)}

    groups = {"position": list(range(0, 9)), "rotation": list(range(9, 18)), "scaling": list(range(18, 27)),
              "opacity": [27, 28], "colour": colour}
    res["blocks_rel"] = {k: rel(blocks[1], blocks[0], rows, seen) for k, rows in groups.items()}
    solved = (flags[0] >= -1).all(0) & (flags[1] >= -1).all(0)
    same = solved & (flags[0] == flags[1]).all(0)
    K = steps[0].shape[0] - gsn.GSN_STEP_BASE
    sgroups = {"position": [0, 1, 2], "rotation": [3], "scaling": [7, 8, 9], "opacity": [10],
               "colour": list(range(gsn.GSN_STEP_BASE, gsn.GSN_STEP_BASE + K))}
    res["steps_rel"] = {k: rel(steps[1], steps[0], rows, same, True) for k, rows in sgroups.items()}
    res["kernels_solved"] = int(solved.sum())
    res["decisions_differ"] = round(float((solved & ~same).sum()) / max(int(solved.sum()), 1), 6)
    res["image"] = int(t)
    return res


def _graph_rate(cfg, targets, dev, order, warmup, steps, step_frac):
    """The plain form with reserved frames, each sweep a replay of its image's captured HIP graph
    (captured before timing), against the same sweeps issued one call at a time (also without host
    waits).  Returns both rates and the device status gathered over the runs."""
    import torch
    out = {}
    for mode in ("eager", "graph"):
        tr = _trainer(cfg, targets, dev, 0, step_frac, reserve=True)
        if mode == "graph":
            for t in sorted(set(int(x) for x in order[:warmup + steps])):
                tr.sweep_graph(t)  # captures, then replays once (untimed)
        for i in range(warmup):
            (tr.sweep_graph if mode == "graph" else tr.sweep)(int(order[i]))
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for i in range(steps):
            (tr.sweep_graph if mode == "graph" else tr.sweep)(int(order[warmup + i]))
        torch.cuda.synchronize(dev)
        el = time.perf_counter() - t0
        stats = tr.check_status()
        tr.close()
        out[mode] = {"value": round(steps / el, 4), "unit": "sweeps/s", "ms_per_step": round(el * 1e3 / steps, 3),
                     "device_status": {k: v for k, v in stats.items() if k != "message"}}
        log(f"[bench] reserved frames, {mode}: {steps / el:.2f} sweeps/s")
    return out


def _sweep_times(tr, order, start, n, learned, dev):
    """Per-sweep wall times (ms) of n more sweeps, each synchronised: median and p10/p90."""
    import numpy as np
    import torch
    ts = []
    for i in range(n):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        _sweep(tr, int(order[start + i]), start + i, learned)
        torch.cuda.synchronize(dev)
        ts.append((time.perf_counter() - t0) * 1e3)
    p10, p50, p90 = np.percentile(ts, [10, 50, 90])
    return {"sweeps": n, "p10_ms": round(float(p10), 3), "median_ms": round(float(p50), 3),
            "p90_ms": round(float(p90), 3)}


def _psnr(tr, targets, dev):
    """Mean PSNR over all training views (images clamped to [0, 1]); evaluation only."""
    import torch

    from paper_2501_13975_amd import gsn
    fr = tr.frames[0]
    vals = []
    for cam, tg in zip(tr.ccams, targets):
        img = torch.empty_like(tg)
        tr.ctx.render(tr.g, cam, tr.ro, fr, img)
        mse = torch.mean((img.clamp(0.0, 1.0) - tg) ** 2)
        vals.append(10.0 * torch.log10(1.0 / mse))
    return float(torch.stack(vals).mean().cpu())


def _curve(tr, nv, max_epochs, checks, step, targets, dev, target=None, first_epoch=0):
    """Sweeps epoch by epoch in the seeded view order, the mean PSNR over all views checked after
    every 1/checks of an epoch.  Returns [(sweeps, seconds of sweeps, psnr)], stopping at the first
    check at or above target when one is given."""
    import numpy as np
    import torch

    from synth.scenes import view_order
    out, spent, i = [], 0.0, 0
    for e in range(first_epoch, first_epoch + max_epochs):
        order = view_order(nv, e)
        bounds = np.linspace(0, nv, checks + 1).astype(int)
        for c in range(checks):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            for t in order[bounds[c]:bounds[c + 1]]:
                step(int(t), i)
                i += 1
            torch.cuda.synchronize(dev)
            spent += time.perf_counter() - t0
            out.append((i, spent, _psnr(tr, targets, dev)))
            if target is not None and out[-1][2] >= target:
                return out
    return out


def _first_crossing(curve, target):
    for sweeps, secs, p in curve:
        if p >= target:
            return sweeps, secs
    return None, None


def _logs(cfg, targets, dev, sweeps, mask, step_frac, seed=0):
    """(features, labels, mask) rows logged by plain full-rule sweeps (the learned form's training
    data), `sweeps` sweeps from the initial state in the seeded view order."""
    from synth.scenes import view_order
    tr = _trainer(cfg, targets, dev, 0, step_frac)
    log = []
    order = view_order(len(cfg.cams), 0)
    for i in range(sweeps):
        tr.log_sweep(int(order[i % len(order)]), log, mask, max_rows=20000, seed=seed + i)
    tr.close()
    return log


def _pretrained(logs, dev, epochs=20):
    """A step-scale network trained by the library's Adam kernels on logged plain sweeps."""
    import torch

    from paper_2501_13975_amd import gsn
    from paper_2501_13975_amd.train import pretrain
    from synth.mlp_init import init_params
    ctx = gsn.Context(dev)
    mlp = gsn.MLP(init_params(0), dev)
    ctx.mlp_reset(mlp)
    curve = pretrain(ctx, mlp, logs, epochs=epochs, batch=8192, lr=1e-2)
    torch.cuda.synchronize(dev)
    ctx.close()
    Lb = torch.cat([x[1] for x in logs], 1)
    M = torch.cat([x[2] for x in logs], 1)
    mean = ((Lb * M).sum(1) / M.sum(1).clamp(min=1)).cpu().numpy()
    return mlp.params.cpu().numpy(), curve, mean


def _equal_psnr(cfg, targets, dev, epochs, every, mask, step_frac, params, label_mean, checks=5):
    """Plain form for `epochs` epochs sets the target PSNR (its value after the last epoch); every form
    is checked after each 1/checks of an epoch and timed to its first check at or above the target
    (sweeps only).  The learned form starts from the pre-trained network; at the learned form's sweep
    count the controls alpha = 1 (the primary-only step) and alpha = the mean logged label run the
    same schedule, to show what the network adds."""
    import numpy as np

    from paper_2501_13975_amd import gsn
    nv = len(cfg.cams)
    out = {"epochs_plain": epochs, "learned_every": every, "group_mask": mask, "step_frac": step_frac,
           "psnr_checks_per_epoch": checks}
    tr = _trainer(cfg, targets, dev, 0, step_frac, reserve=True)
    out["initial_psnr"] = round(_psnr(tr, targets, dev), 4)
    pc = _curve(tr, nv, epochs, checks, lambda t, i: tr.sweep(t, mask), targets, dev)
    tr.close()
    target = pc[-1][2]
    ps, psec = _first_crossing(pc, target)
    out.update(target_psnr=round(target, 4), plain_curve=[round(x[2], 3) for x in pc], plain_sweeps=ps,
               plain_seconds=round(psec, 3))
    log(f"[bench] plain: target {target:.3f} dB after {pc[-1][0]} sweeps; first reached after {ps} ({psec:.2f}s)")
    runs = {}
    for mode in ("mlp", "one", "const"):
        tr = _trainer(cfg, targets, dev, 0, step_frac, reserve=True)
        tr.enable_learned(None, every=every, lr=1e-2, alpha_mode=mode, alpha_const=float(np.mean(label_mean)),
                          mlp=_mlp_from(params, dev, tr))
        step = lambda t, i: tr.sweep_learned(t, i, mask)  # noqa: E731
        if mode == "mlp":
            lc = _curve(tr, nv, 3 * epochs, checks, step, targets, dev, target=target)
            ls, lsec = _first_crossing(lc, target)
            runs[mode] = {"curve": [round(x[2], 3) for x in lc], "sweeps": lc[-1][0], "seconds": round(lc[-1][1], 3),
                          "psnr": round(lc[-1][2], 4), "reached_target": ls is not None,
                          "mean_abs_alpha_error": tr.learned_error(), "fallback_sweeps": tr.fallback_sweeps}
            budget = lc[-1][0]
        else:
            # the same number of sweeps as the network's run, same schedule of full-rule sweeps
            from synth.scenes import view_order
            i = 0
            for e in range(3 * epochs):
                for t in view_order(nv, e):
                    if i >= budget:
                        break
                    tr.sweep_learned(int(t), i, mask)
                    i += 1
            runs[mode] = {"sweeps": i, "psnr": round(_psnr(tr, targets, dev), 4)}
        tr.close()
        log(f"[bench] learned form, alpha {mode}: {runs[mode]}")
    out["learned"] = runs["mlp"]
    out["controls_at_equal_sweeps"] = {"alpha_one": runs["one"], "alpha_mean_label": runs["const"],
                                       "alpha_mean_label_value": [round(float(x), 4) for x in label_mean]}
    out["speedup_at_equal_psnr"] = (round(psec / runs["mlp"]["seconds"], 3) if runs["mlp"]["reached_target"]
                                    else None)
    return out


def _mlp_from(params, dev, tr):
    """A fresh network state (zero Adam moments) with the given master weights."""
    from paper_2501_13975_amd import gsn
    m = gsn.MLP(params, dev)
    tr.ctx.mlp_reset(m)
    return m


def _c4_leg(dev, every, mask, step_frac, params, label_mean, epochs=1):
    """The largest configuration: 3M kernels, 300 cameras at 1920x1080 (3 half-resolution
    secondaries), plain form against the learned form started from the network pre-trained on
    logged plain sweeps of the smaller scenes, timed to equal PSNR."""
    from synth.scenes import make_config
    t0 = time.time()
    cfg = make_config("c4")
    targets = _targets(cfg, dev)
    log(f"[bench] c4: {cfg.n} kernels, {len(cfg.cams)} cameras ready ({time.time() - t0:.1f}s)")
    out = _equal_psnr(cfg, targets, dev, epochs, every, mask, step_frac, params, label_mean)
    out["workload"] = (f"{cfg.n} Gaussians SH3, {len(cfg.cams)} cameras at {cfg.width}x{cfg.height}, "
                       f"{cfg.n_secondary} half-resolution secondaries")
    del targets
    return out


def _variant_rates(cfg, targets, dev, order, warmup, steps, step_frac):
    """Sweep rate of the plain form on the benchmark workload with |N_t| = 0 and 8 secondaries
    (Sec. 4.3) and with the local Gauss-Newton blocks at |N_t| = 3."""
    out = {}
    for name, K, gn in (("secondaries_0", 0, False), ("secondaries_8", 8, False), ("gauss_newton", None, True)):
        tr = _trainer(cfg, targets, dev, 0, step_frac, n_secondary=K, gauss_newton=gn)
        el, st, cn = _rate_and_profile(tr, order, warmup, steps, False, dev)
        tr.close()
        out[name] = {"value": round(steps / el, 4), "unit": "sweeps/s", "ms_per_step": round(el * 1e3 / steps, 3),
                     "stage_ms_per_step": {k: round(v[0] / steps, 3) for k, v in st.items()},
                     "counts_per_step": {k: int(v / steps) for k, v in cn.items()}}
        log(f"[bench] {name}: {steps / el:.2f} sweeps/s")
    return out


def _overshoot_leg(dev, epochs, mask, step_frac):
    """|N_t| ablation and the Gauss-Newton variant on the 100k-kernel, 50-camera 1024x768 scene.

    Overshoot at a view switch (Sec. 4.3): for every sweep on image t, the relative change of
    the L2 loss of the image trained next (t') across the sweep, (L_t'(after) - L_t'(before)) /
    L_t'(before); a spike is a sweep that raises it.  Also the primary's own relative change,
    the mean PSNR over all views after the epochs and the seconds spent in sweeps."""
    import numpy as np
    import torch

    from synth.scenes import make_config, view_order
    cfg = make_config("c1")
    targets = _targets(cfg, dev)
    nv = len(cfg.cams)
    out = {"workload": (f"{cfg.n} Gaussians SH3, {nv} cameras at {cfg.width}x{cfg.height}, "
                        f"secondaries at half resolution"),
           "epochs": epochs, "group_mask": mask, "step_frac": step_frac, "runs": {}}
    for name, K, gn in (("secondaries_0", 0, False), ("secondaries_3", 3, False), ("secondaries_8", 8, False),
                        ("gauss_newton_3", 3, True)):
        tr = _trainer(cfg, targets, dev, 0, step_frac, n_secondary=K, gauss_newton=gn)
        img = torch.empty_like(targets[0])

        def l2(v):
            tr.ctx.render(tr.g, tr.ccams[v], tr.ro, tr.frames[0], img)
            return torch.mean((img - targets[v]) ** 2)

        p0 = _psnr(tr, targets, dev)
        rows, spent = [], 0.0
        for e in range(epochs):
            order = view_order(nv, e)
            for i, t in enumerate(order):
                t, nxt = int(t), int(order[(i + 1) % nv])
                before = torch.stack([l2(t), l2(nxt)])
                torch.cuda.synchronize(dev)
                t0 = time.perf_counter()
                tr.sweep(t, mask)
                torch.cuda.synchronize(dev)
                spent += time.perf_counter() - t0
                rows.append(torch.cat([before, torch.stack([l2(t), l2(nxt)])]))
        r = torch.stack(rows).double().cpu().numpy()
        prim = (r[:, 2] - r[:, 0]) / r[:, 0]
        nxt = (r[:, 3] - r[:, 1]) / r[:, 1]
        psnr = _psnr(tr, targets, dev)
        tr.close()
        out["runs"][name] = {"secondaries": K, "gauss_newton": gn, "sweeps": len(r),
                             "psnr_initial": round(p0, 4), "psnr_final": round(psnr, 4),
                             "primary_rel_change_mean": round(float(prim.mean()), 6),
                             "next_view_rel_change_mean": round(float(nxt.mean()), 6),
                             "next_view_rel_change_p90": round(float(np.percentile(nxt, 90)), 6),
                             "spike_fraction": round(float((nxt > 0).mean()), 4),
                             "sweep_seconds": round(spent, 3)}
        log(f"[bench] overshoot {name}: {out['runs'][name]}")
    return out


def _order_leg(dev, epochs, step_frac):
    """Schedules and optimisation order on the 100k-kernel, 50-camera 1024x768 scene (Sec. 4.2,
    Sec. 5): every group trained, for `epochs` epochs, by the jacobi sweep, by the series sweep
    in the paper's order (position, rotation, scaling, opacity, colour) and by the series sweep
    in the reverse order (colour first).  Mean PSNR over all views and seconds of sweeps."""
    import torch

    from synth.scenes import make_config, view_order
    cfg = make_config("c1")
    targets = _targets(cfg, dev)
    nv = len(cfg.cams)
    out = {"workload": f"{cfg.n} Gaussians SH3, {nv} cameras at {cfg.width}x{cfg.height}, 3 secondaries",
           "epochs": epochs, "step_frac": step_frac, "runs": {}}
    for name, order in (("jacobi", None), ("series_p_q_s_o_c", (1, 2, 4, 8, 16)),
                        ("series_c_o_s_q_p", (16, 8, 4, 2, 1))):
        tr = _trainer(cfg, targets, dev, 0, step_frac)
        p0 = _psnr(tr, targets, dev)
        spent, curve = 0.0, []
        for e in range(epochs):
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            for t in view_order(nv, e):
                if order is None:
                    tr.sweep(int(t), 31)
                else:
                    tr.sweep_series(int(t), order)
            torch.cuda.synchronize(dev)
            spent += time.perf_counter() - t0
            curve.append(round(_psnr(tr, targets, dev), 4))
        tr.close()
        out["runs"][name] = {"psnr_initial": round(p0, 4), "psnr_per_epoch": curve, "sweep_seconds": round(spent, 3)}
        log(f"[bench] order {name}: {out['runs'][name]}")
    return out


# Adam learning rates of the first-order baseline (position, rotation, linear scale, opacity, SH):
# the usual 3DGS rates carried over to these parameterisations (log-scale 5e-3 at s ~ 0.02, logit
# opacity 0.05 at sigma ~ 0.5).
ADAM_LR = (1.6e-4, 1e-3, 1e-4, 1.25e-2, 2.5e-3)


def _first_order_leg(dev, newton_epochs, max_epochs, mask, step_frac, checks=5):
    """Newton sweeps against Adam iterations on the same gradients, 100k-kernel scene (Sec. 1
    and Sec. 5 claim far fewer Newton iterations than first-order ones).  The Newton form
    (jacobi, 3 secondaries) trains `newton_epochs` epochs and sets the target PSNR (its value after
    the last epoch); Adam (the primary view's gradient, one image per iteration) runs with the
    learning rates ADAM_LR scaled by 0.3, 1 and 3 until it reaches the target or `max_epochs`
    epochs.  Every form is checked after each 1/checks of an epoch; iterations and seconds are taken
    at the first check at or above the target."""
    from synth.scenes import make_config
    cfg = make_config("c1")
    targets = _targets(cfg, dev)
    nv = len(cfg.cams)
    out = {"workload": f"{cfg.n} Gaussians SH3, {nv} cameras at {cfg.width}x{cfg.height}",
           "group_mask": mask, "newton_step_frac": step_frac, "adam_lr": list(ADAM_LR), "psnr_checks_per_epoch": checks}
    tr = _trainer(cfg, targets, dev, 0, step_frac)
    out["psnr_initial"] = round(_psnr(tr, targets, dev), 4)
    nc = _curve(tr, nv, newton_epochs, checks, lambda t, i: tr.sweep(t, mask), targets, dev)
    tr.close()
    target = nc[-1][2]
    ns, nsec = _first_crossing(nc, target)
    out["newton"] = {"curve": [round(x[2], 4) for x in nc], "psnr": round(target, 4), "sweeps_to_target": ns,
                     "seconds_to_target": round(nsec, 4)}
    runs = {}
    for f in (0.3, 1.0, 3.0):
        lr = [x * f for x in ADAM_LR]
        tr = _trainer(cfg, targets, dev, 0, 1.0, n_secondary=0)
        ac = _curve(tr, nv, max_epochs, checks,
                    lambda t, i: tr.sweep_first_order(t, lr, adam=True, group_mask=mask), targets, dev, target=target)
        tr.close()
        its, secs = _first_crossing(ac, target)
        runs[f"lr_x{f:g}"] = {"curve": [round(x[2], 4) for x in ac], "iterations_to_target": its,
                              "seconds_to_target": None if secs is None else round(secs, 4),
                              "best_psnr": round(max(x[2] for x in ac), 4)}
        log(f"[bench] adam lr x{f:g}: {runs[f'lr_x{f:g}']}")
    out["adam"] = runs
    best = [r for r in runs.values() if r["iterations_to_target"]]
    if best:
        b = min(best, key=lambda r: r["iterations_to_target"])
        out["iterations_ratio"] = round(b["iterations_to_target"] / ns, 3)
        out["seconds_ratio"] = round(min(r["seconds_to_target"] for r in best) / nsec, 3)
    else:
        out["iterations_ratio"] = out["seconds_ratio"] = None
    log(f"[bench] first-order vs Newton: {out}")
    return out


def _psnr_curve_leg(dev, epochs, mask, step_frac):
    """Mean PSNR over all views after each epoch of the plain form on the 100k-kernel, 50-camera
    1024x768 scene (jacobi, 3 secondaries)."""
    import torch

    from synth.scenes import make_config, view_order
    cfg = make_config("c1")
    targets = _targets(cfg, dev)
    nv = len(cfg.cams)
    tr = _trainer(cfg, targets, dev, 0, step_frac)
    out = {"workload": f"{cfg.n} Gaussians SH3, {nv} cameras at {cfg.width}x{cfg.height}, 3 secondaries",
           "group_mask": mask, "step_frac": step_frac, "psnr_initial": round(_psnr(tr, targets, dev), 4),
           "psnr_per_epoch": [], "seconds_per_epoch": []}
    for e in range(epochs):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for t in view_order(nv, e):
            tr.sweep(int(t), mask)
        torch.cuda.synchronize(dev)
        out["seconds_per_epoch"].append(round(time.perf_counter() - t0, 4))
        out["psnr_per_epoch"].append(round(_psnr(tr, targets, dev), 4))
    tr.close()
    log(f"[bench] PSNR curve: {out}")
    return out


def _batched_solve_leg(dev, reps=20):
    """The eight scenes of 20k-800k kernels at 1280x720: blocks from one primary and three
    secondary views each, then the solves of all scenes timed as one launch per scene, as
    one batched launch (autotuned shape) and as a replayed HIP graph."""
    import numpy as np
    import torch

    from paper_2501_13975_amd import gsn
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    from synth.scenes import C3_SIZES, make_config
    trs, items, total = [], [], 0
    for i in range(len(C3_SIZES)):
        cfg = make_config(f"c3_{i}")
        targets = _targets(cfg, dev)
        g = gsn.DeviceGaussians.from_host(cfg.init, dev)
        tr = LocalNewtonTrainer(g, cfg.cams, targets, n_secondary=cfg.n_secondary)
        tr.accumulate(0)
        trs.append(tr)
        items.append((tr.g, tr.ccams[0], tr.blocks, tr.solve_opts(0), tr.steps))
        total += cfg.n
    torch.cuda.synchronize(dev)
    ctx = trs[0].ctx

    def timed(fn):
        fn()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize(dev)
        return (time.perf_counter() - t0) * 1e3 / reps

    per_scene = timed(lambda: [tr.ctx.local_newton_solve(*it[:4], it[4]) for tr, it in zip(trs, items)])
    block, grid = ctx.solve_tune(items)
    batched = timed(lambda: ctx.solve_batched(items))
    graph = ctx.solve_graph(items)
    graphed = timed(graph.launch)
    graph.close()
    for tr in trs:
        tr.close()
    return {"scenes": len(C3_SIZES), "kernels": total, "views": "1280x720 + 3 half-resolution secondaries",
            "ms_per_scene_launches": round(per_scene, 4), "ms_batched": round(batched, 4),
            "ms_graph": round(graphed, 4), "tuned_block": block, "tuned_grid": grid,
            "kernels_solved_per_s_graph": round(total / (graphed * 1e-3), 1)}


def gpu_run(args):
    import numpy as np
    import torch

    from synth.scenes import make_config, view_order

    t0 = time.time()
    cfg = make_config(args.config)
    dev = torch.device("cuda", 0)
    log(f"[bench] generated {args.config}: {cfg.n} kernels, {len(cfg.cams)} cameras ({time.time() - t0:.1f}s)")
    targets = _targets(cfg, dev)
    log(f"[bench] rendered {len(targets)} targets ({time.time() - t0:.1f}s)")
    order = np.concatenate([view_order(len(cfg.cams), e) for e in range(8)])
    tr = _trainer(cfg, targets, dev, 0, args.step_frac, reserve=True)
    # the rate: sweeps without profiling; then the same number of sweeps, profiled, for the stage
    # times, the work counters and the roofline of the dominant kernel
    elapsed, _, _ = _timed(tr, order, args.warmup, args.steps, False, dev, profile=False)
    prof_el, stages, counts = _timed(tr, order[args.warmup + args.steps:], 0, args.steps, False, dev)
    log(f"[bench] plain: {args.steps / elapsed:.2f} sweeps/s; profiled {args.steps / prof_el:.2f} sweeps/s")
    dist = _sweep_times(tr, order, args.warmup + 2 * args.steps, 30, False, dev)
    # the raster passes' lane use, from a few more sweeps that also count their wave steps
    _, _, lane_counts = _timed(tr, order[args.warmup + 2 * args.steps + 30:], 0, 8, False, dev, wave_steps=True)
    status = tr.check_status()
    tr.close()
    graph = _graph_rate(cfg, targets, dev, order, args.warmup, args.steps, args.step_frac) if args.graph_leg else None
    log(f"[bench] plain: {args.steps} sweeps in {elapsed:.3f}s; stage ms: "
        + ", ".join(f"{k}={v[0]:.1f}" for k, v in stages.items()))
    # the mixed precision form alone (full rule every sweep), then with the learned step scale
    tr = _trainer(cfg, targets, dev, 0, args.step_frac, reserve=True, precision=1)
    el_m, st_m, _ = _rate_and_profile(tr, order, args.warmup, args.steps, False, dev)
    tr.close()
    mixed = {"value": round(args.steps / el_m, 4), "unit": "sweeps/s", "ms_per_step": round(el_m * 1e3 / args.steps, 3),
             "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in st_m.items()}}
    log(f"[bench] mixed: {args.steps / el_m:.2f} sweeps/s; stage ms: "
        + ", ".join(f"{k}={v[0]:.1f}" for k, v in st_m.items()))
    mixed["vs_plain"] = _mixed_vs_plain(cfg, targets, dev, int(order[0]), args.step_frac)
    log(f"[bench] mixed against plain: {mixed['vs_plain']}")
    learned = None
    if args.learned_every:
        tr = _trainer(cfg, targets, dev, args.learned_every, args.step_frac, reserve=True)
        el2, st2, _ = _rate_and_profile(tr, order, args.warmup, args.steps, True, dev)
        tr.close()
        learned = {"value": round(args.steps / el2, 4), "unit": "sweeps/s", "ms_per_step": round(el2 * 1e3 / args.steps, 3),
                   "every": args.learned_every,
                   "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in st2.items()}}
        log(f"[bench] learned: {args.steps} sweeps in {el2:.3f}s")
    variants = None
    if args.variants_leg:
        variants = _variant_rates(cfg, targets, dev, order, args.warmup, args.steps, args.step_frac)
    overshoot = None
    if args.overshoot_epochs > 0:
        overshoot = _overshoot_leg(dev, args.overshoot_epochs, args.quality_mask, args.quality_step_frac)
    order_exp = None
    if args.order_epochs > 0:
        order_exp = _order_leg(dev, args.order_epochs, args.order_step_frac)
    curve = None
    if args.curve_epochs > 0:
        curve = _psnr_curve_leg(dev, args.curve_epochs, args.quality_mask, args.quality_step_frac)
    first_order = None
    if args.first_order_epochs > 0:
        first_order = _first_order_leg(dev, 1, args.first_order_epochs, args.quality_mask, args.quality_step_frac)
    batched = None
    if args.batched_leg:
        batched = _batched_solve_leg(dev)
        log(f"[bench] batched solve: {batched}")
    quality = c4 = pre = None
    if args.quality_epochs > 0 and args.learned_every:
        # the network learns from (features, alpha_eff) rows that plain sweeps log on the 100k scene and
        # on this workload, before any timed run
        from synth.scenes import make_config as _mk
        c1 = _mk("c1")
        t1 = _targets(c1, dev)
        logs = _logs(c1, t1, dev, len(c1.cams), args.quality_mask, args.quality_step_frac)
        del t1
        logs += _logs(cfg, targets, dev, args.log_sweeps, args.quality_mask, args.quality_step_frac, seed=1000)
        params, pcurve, label_mean = _pretrained(logs, dev)
        pre = {"rows": int(sum(x[0].shape[1] for x in logs)), "loss_per_epoch": [round(x, 5) for x in pcurve],
               "sources": f"{len(c1.cams)} plain sweeps of the 100k scene, {args.log_sweeps} of this workload",
               "mean_label": [round(float(x), 4) for x in label_mean]}
        log(f"[bench] pre-trained the step-scale network: {pre}")
        del logs
        quality = _equal_psnr(cfg, targets, dev, args.quality_epochs, args.learned_every, args.quality_mask,
                              args.quality_step_frac, params, label_mean)
        if args.c4_epochs > 0:
            del targets
            c4 = _c4_leg(dev, args.learned_every, args.quality_mask, args.quality_step_frac, params, label_mean,
                         args.c4_epochs)
    return dict(elapsed=elapsed, stages=stages, counts=counts, lane_counts=lane_counts, cfg=cfg, mixed=mixed, learned=learned, quality=quality,
                batched=batched, variants=variants, overshoot=overshoot, order_exp=order_exp,
                first_order=first_order, dist=dist, curve=curve, graph=graph, status=status, c4=c4, pre=pre)


def _measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when the
    kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_c2_traffic.txt")
    if not os.path.exists(path):
        return None
    d = json.loads(open(path).read())
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in d["sources"])
    if hashlib.sha256(src).hexdigest() != d["source_sha256"]:
        return None
    return d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]


def copy_bandwidth(dev, nbytes=1 << 30, reps=5):
    """Measured device-to-device copy bandwidth (read + write bytes per second), GB/s."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize(dev)
    el = time.perf_counter() - t0
    del a, b
    return 2.0 * nbytes * reps / el / 1e9


def copy_probe(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes x{reps}", flush=True)


def sweep_roofline(value, counts, steps, n, views, pixels_per_step, copy_gbs):
    """The whole sweep against HBM: the bytes the method must move per sweep,
    N (708 + 384 V) per kernel set + 28 per emitted pair + 40 per list entry the forward pass
    consumes + 40 per entry the backward pass consumes + 112 per pixel, times sweeps/s, against the
    8 TB/s peak and a measured copy."""
    b_alg = (n * (708 + 384 * views) + BYTES_PAIR * counts["pairs"] / steps
             + BYTES_ENTRY * (counts["fwd_staged"] + counts["bwd_staged"]) / steps + 112.0 * pixels_per_step)
    gbs = b_alg * value / 1e9
    return {"algorithmic_bytes_per_sweep": round(b_alg), "achieved": round(gbs, 1), "unit": "GB/s",
            "peak": PEAK_HBM_GBS, "frac": round(gbs / PEAK_HBM_GBS, 5),
            "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(gbs / copy_gbs, 5)}


def roofline(stages, counts, steps, pixels_per_step, n, views):
    """Roofline figure of the stage that takes the most time (one kernel per raster stage launch):
    algorithmic FLOPs and bytes per launch from the work counters, over the launch's average time
    (HIP events on the library's stream).  The raster passes report the ALU bound (against the
    published FP32 vector peak, with the unpacked rate beside it) and their HBM fraction."""
    dom = max(stages, key=lambda s: stages[s][0])
    ms, launches = stages[dom]
    launches = max(launches, 1)
    per_launch_s = ms * 1e-3 / launches
    out = dict(kernel=dom, avg_launch_ms=round(ms / launches, 4), launches=launches)
    if dom in ("raster_bwd", "raster_fwd"):
        if dom == "raster_bwd":
            flops = FLOP_EVAL * counts["bwd_evals"] + FLOP_BWD_PAIR * counts["bwd_active"]
            nbytes = (BYTES_ENTRY * counts["bwd_staged"] + BYTES_BWD_PIXEL * pixels_per_step * steps
                      + BYTES_ZSTATS * n * views * steps)
        else:
            flops = FLOP_EVAL * counts["fwd_evals"] + FLOP_FWD_BLEND * counts["bwd_active"]
            nbytes = BYTES_ENTRY * counts["fwd_staged"] + BYTES_FWD_PIXEL * pixels_per_step * steps
        achieved = flops / launches / per_launch_s / 1e12
        traffic = _measured_traffic(dom)
        alg_bytes = nbytes / launches
        out.update(bound="alu", achieved=round(achieved, 3), peak=PEAK_ALU_TFLOPS, unit="TFLOP/s",
                   frac=round(achieved / PEAK_ALU_TFLOPS, 5), traffic=traffic,
                   peak_unpacked=PEAK_ALU_UNPACKED_TFLOPS, frac_unpacked=round(achieved / PEAK_ALU_UNPACKED_TFLOPS, 5),
                   algorithmic_flops_per_launch=round(flops / launches),
                   algorithmic_bytes_per_launch=round(alg_bytes),
                   hbm_achieved_gbs=round(alg_bytes / per_launch_s / 1e9, 1),
                   hbm_fraction=round(alg_bytes / per_launch_s / 1e9 / PEAK_HBM_GBS, 5),
                   algorithmic_bytes_within_traffic=(None if traffic is None else bool(alg_bytes <= traffic)))
        if traffic is not None and alg_bytes > traffic:
            log(f"[bench] WARNING: {dom} algorithmic bytes {alg_bytes:.3e} exceed the measured traffic {traffic:.3e}")
        return out
    # sort/bin: 28 algorithmic bytes per (tile, kernel) pair (write key/value, read per tile, write list)
    nbytes = BYTES_PAIR * counts["pairs"]
    achieved = nbytes / launches / per_launch_s / 1e9
    out.update(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
               frac=round(achieved / PEAK_HBM_GBS, 5), traffic=None)
    return out


def lane_use(c):
    """Share of a wave's 64 lanes at work in the raster passes' per-pixel loops: per-pixel steps
    over 64 x the waves' steps (counted in sweeps profiled at level 2)."""
    cyc = [c[f"bwd_cycles_{p}"] for p in ("stage", "scan", "walk", "sums")]
    tot = max(sum(cyc), 1)
    return {"fwd": round(c["fwd_evals"] / max(64 * c["fwd_wave_steps"], 1), 3),
            "bwd": round((c["bwd_active"] + c["bwd_evals"]) / max(64 * c["bwd_wave_steps"], 1), 3),
            "bwd_wave_time_share": {p: round(x / tot, 3) for p, x in zip(("stage", "scan", "walk", "sums"), cyc)},
            "sweeps": 8}


def solve_rules(counts):
    """How often each of the solve's safeguards bound, per solved kernel (a kernel's group is
    counted once per sweep): damping escalated, gradient fallback, trust radius, opacity bounds."""
    solved = max(counts.get("solved", 0), 1)
    out = {"kernels_solved": counts.get("solved", 0)}
    for g in ("position", "rotation", "scaling", "opacity"):
        out[f"escalated_{g}"] = round(counts[f"escalated_{g}"] / solved, 6)
        out[f"fallback_{g}"] = round(counts[f"fallback_{g}"] / solved, 6)
    for g in ("position", "rotation", "scaling", "colour"):
        out[f"trust_clamped_{g}"] = round(counts[f"clamped_{g}"] / solved, 6)
    out["opacity_bound"] = round(counts["opacity_bound"] / solved, 6)
    return out


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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--learned-every", type=int, default=4,
                    help="learned form: one full-rule (training) sweep every N sweeps; 0 skips the learned form")
    ap.add_argument("--quality-epochs", type=int, default=2,
                    help="epochs of the plain form that set the PSNR both forms are timed to; 0 skips")
    ap.add_argument("--step-frac", type=float, default=0.002,
                    help="fraction of every Newton step applied in the timed sweeps: the full step is computed, "
                         "and a small fraction keeps the scene near its initial state so that every timed sweep "
                         "sees the same workload")
    ap.add_argument("--c4-epochs", type=int, default=1,
                    help="epochs of the plain form on the 3M-kernel, 300-camera workload that set its equal-PSNR "
                         "target; 0 skips")
    ap.add_argument("--log-sweeps", type=int, default=20,
                    help="plain sweeps of this workload logged for the network's pre-training")
    ap.add_argument("--no-overlap", action="store_true",
                    help="the paper's plain steps: no overlap-share scaling of the simultaneous kernel steps")
    ap.add_argument("--quality-mask", type=int, default=31,
                    help="attribute groups trained in the equal-PSNR leg (bits: 1 position, 2 rotation, 4 scaling, "
                         "8 opacity, 16 colour)")
    ap.add_argument("--quality-step-frac", type=float, default=1.0)
    ap.add_argument("--no-batched-leg", dest="batched_leg", action="store_false",
                    help="skip timing the batched solve of the eight 20k-800k scenes")
    ap.add_argument("--no-graph-leg", dest="graph_leg", action="store_false",
                    help="skip timing the plain form as replayed HIP graphs of whole sweeps")
    ap.add_argument("--no-variants-leg", dest="variants_leg", action="store_false",
                    help="skip timing |N_t| = 0, 8 and the Gauss-Newton blocks on the benchmark workload")
    ap.add_argument("--overshoot-epochs", type=int, default=1,
                    help="epochs of the |N_t| / Gauss-Newton overshoot comparison on the 100k scene; 0 skips")
    ap.add_argument("--order-epochs", type=int, default=1,
                    help="epochs of the jacobi / series-order comparison on the 100k scene; 0 skips")
    ap.add_argument("--order-step-frac", type=float, default=1.0,
                    help="step fraction of the order comparison (it trains every group)")
    ap.add_argument("--curve-epochs", type=int, default=10,
                    help="epochs of the plain-form PSNR curve on the 100k scene; 0 skips")
    ap.add_argument("--first-order-epochs", type=int, default=10,
                    help="at most this many epochs of Adam against one epoch of Newton sweeps on the 100k "
                         "scene; 0 skips")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB on the device three times and exit (the calibration run of the HBM "
                         "traffic counters)")
    args = ap.parse_args()
    global OVERLAP
    OVERLAP = 0 if args.no_overlap else 1
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the training step runs on a single MI355X; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    r = gpu_run(args)
    elapsed, stages, counts, cfg, status = r["elapsed"], r["stages"], r["counts"], r["cfg"], r["status"]
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.steps / elapsed
    pixels = cfg.width * cfg.height + cfg.n_secondary * (cfg.width // 2) * (cfg.height // 2)
    rl = roofline(stages, counts, args.steps, pixels, cfg.n, 1 + cfg.n_secondary)
    import torch
    srl = sweep_roofline(value, counts, args.steps, cfg.n, 1 + cfg.n_secondary, pixels,
                         copy_bandwidth(torch.device("cuda", 0)))
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
                   "secondaries": cfg.n_secondary, "form": "plain", "step_frac": args.step_frac},
        "gaussians_updated_per_s": round(value * cfg.n, 1),
        "sweep_ms_distribution": r["dist"],
        "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
        "counts_per_step": {k: int(v / args.steps) for k, v in counts.items()},
        # share of a wave's 64 lanes at work in the raster passes' per-pixel loops
        "raster_lane_use": lane_use(r["lane_counts"]),
        "roofline": rl,
        "sweep_hbm": srl,
        "solve_rules": solve_rules({k: v / args.steps for k, v in counts.items()}),
        "device_status": {k: v for k, v in status.items() if k != "message"},
        "reserved_graph": r["graph"],
        "cpu_baseline": cpu,
        "mixed": r["mixed"],
        "learned": r["learned"],
        "equal_psnr": r["quality"],
        "learned_pretraining": r["pre"],
        "c4_equal_psnr": r["c4"],
        "batched_solve": r["batched"],
        "variants": r["variants"],
        "overshoot": r["overshoot"],
        "schedule_order": r["order_exp"],
        "first_order": r["first_order"],
        "psnr_curve": r["curve"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
