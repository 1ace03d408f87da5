"""Stochastic local-Newton training loop on the GPU (Sec. 4.1-4.3).

One sweep trains on one image t (the primary target): render and accumulate
its blocks, render and accumulate each of its K nearest cameras at half
resolution (secondary targets, overshoot control), solve every kernel's local
Newton systems and apply the steps.  All of it runs in libgsn; this class owns
the device buffers and issues the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gsn


class LocalNewtonTrainer:
    def __init__(self, gauss: gsn.DeviceGaussians, cams, targets, n_secondary=3, lambda_ssim=0.2,
                 render_opts=None, solve_kw=None, device="cuda", keep_zstats=False):
        self.g = gauss
        self.dev = torch.device(device)
        self.ctx = gsn.Context(self.dev)
        self.cams = list(cams)
        self.ccams = [gsn.camera(c) for c in self.cams]
        self.half = [c.downsampled() for c in self.cams]
        self.chalf = [gsn.camera(c) for c in self.half]
        self.targets = targets
        self.n_secondary = int(n_secondary) if len(self.cams) > 1 else 0
        self.ro = render_opts or gsn.render_opts()
        self.lo = gsn.loss_opts(lambda_ssim, 1.0, keep_zstats)
        self.solve_kw = dict(solve_kw or {})
        V = 1 + self.n_secondary
        self.blocks = gsn.Blocks(gauss.n, V, self.dev)
        self.steps = gsn.Steps(gauss.n, gauss.sh_degree, self.dev)
        self.frames = [self.ctx.frame() for _ in range(V)]
        self.loss = torch.zeros(V, 2, dtype=torch.float64, device=self.dev)
        if self.n_secondary:
            centers = np.stack([c.center for c in self.cams])
            scene_center = gauss.pos.double().mean(dim=1).cpu().numpy()
            self.knn = gsn.camera_knn(centers, scene_center, self.n_secondary)
            self.half_targets = []
            for c, tg in zip(self.cams, targets):
                d = torch.empty(3, c.height // 2, c.width // 2, dtype=torch.float32, device=self.dev)
                self.ctx.downsample2x(tg, c.width, c.height, d)
                self.half_targets.append(d)
        else:
            self.knn = np.zeros((len(self.cams), 0), np.int32)
            self.half_targets = []

    def solve_opts(self, t):
        c = self.cams[t]
        return gsn.solve_opts(c.width * c.height, kappa=self.ro.kappa, **self.solve_kw)

    def accumulate(self, t):
        """Primary and secondary renders and block accumulation for training image t."""
        self.ctx.blocks_zero(self.blocks)
        views = [(self.ccams[t], self.targets[t])]
        for j in self.knn[t]:
            views.append((self.chalf[j], self.half_targets[j]))
        for slot, (cam, tgt) in enumerate(views):
            fr = self.frames[slot]
            self.ctx.render(self.g, cam, self.ro, fr)
            self.ctx.accumulate_hessian(self.g, fr, tgt, self.lo, slot, self.blocks, self.loss[slot])

    def sweep(self, t, group_mask=31):
        self.accumulate(t)
        so = self.solve_opts(t)
        self.ctx.local_newton_solve(self.g, self.ccams[t], self.blocks, so, self.steps)
        self.ctx.apply_step(self.g, self.steps, so, group_mask)

    def close(self):
        for f in self.frames:
            f.close()
        self.ctx.close()
