"""Stochastic local-Newton training loop on the GPU (Sec. 4.1-4.3).

One sweep trains on one image t (the primary target): render and accumulate
its blocks, render and accumulate each of its K nearest cameras at half
resolution (secondary targets, overshoot control), solve every kernel's local
Newton systems and apply the steps.  All of it runs in libgsn; this class owns
the device buffers and issues the calls.

Learned form (``enable_learned``): every ``every``-th sweep runs the full rule
and also trains the step-scale network on it (labels: how much of the
primary-only step the full-rule step keeps, per kernel and group); the other
sweeps render only the primary view and scale its Newton step by the network's
prediction.  A learned sweep on which some kernel's features leave the trained
range falls back to the full rule (and trains on it).

Reserved frames (``reserve_frames``) keep every buffer at a fixed size, so a
sweep never waits for the device; ``sweep_graph`` then replays a captured sweep
(one HIP graph per training image and group mask).  ``check_status`` reads what
the device met meanwhile (non-finite kernels culled or skipped, pair-capacity
overflows, after which the frames are reserved again with room for the view).
"""
from __future__ import annotations

import numpy as np
import torch

from . import gsn


class LocalNewtonTrainer:
    def __init__(self, gauss: gsn.DeviceGaussians, cams, targets, n_secondary=3, lambda_ssim=0.2,
                 render_opts=None, solve_kw=None, device="cuda", keep_zstats=False, gauss_newton=False):
        self.g = gauss
        self.dev = torch.device(device)
        self.ctx = gsn.Context(self.dev)
        self.cams = list(cams)
        self.ccams = [gsn.camera(c) for c in self.cams]
        self.chalf = [gsn.camera_half(c) for c in self.ccams]
        self.targets = targets
        self.n_secondary = int(n_secondary) if len(self.cams) > 1 else 0
        self.solve_kw = dict(solve_kw or {})
        # the mixed form (solve precision 1) also accumulates in single precision; its colour sums along
        # each ray stay in double (in single precision they move the position and rotation steps by ~1e-4)
        mixed = int(self.solve_kw.get("precision", 0) == 1)
        self.ro = render_opts or gsn.render_opts()
        self.lo = gsn.loss_opts(lambda_ssim, 1.0, keep_zstats, gauss_newton, precision=mixed)
        V = 1 + self.n_secondary
        self.blocks = gsn.Blocks(gauss.n, V, self.dev)
        self.steps = gsn.Steps(gauss.n, gauss.sh_degree, self.dev)
        self.frames = [self.ctx.frame() for _ in range(V)]
        self.loss = torch.zeros(V, 2, dtype=torch.float64, device=self.dev)
        if self.n_secondary:
            centers = np.stack([c.center for c in self.cams])
            sc = torch.zeros(3, dtype=torch.float64, device=self.dev)
            self.ctx.scene_center(gauss, sc)
            self.knn = gsn.camera_knn(centers, sc.cpu().numpy(), self.n_secondary)
            self.half_targets = []
            for c, tg in zip(self.cams, targets):
                d = torch.empty(3, c.height // 2, c.width // 2, dtype=torch.float32, device=self.dev)
                self.ctx.downsample2x(tg, c.width, c.height, d)
                self.half_targets.append(d)
        else:
            self.knn = np.zeros((len(self.cams), 0), np.int32)
            self.half_targets = []

    # ------------------------------------------------------- reserved frames, graphs
    def reserve_frames(self, margin=1.25, extra=1 << 16):
        """Sizes every frame for the largest pair count any training view needs at the current state
        (primary slot: full resolution; secondary slots: half resolution) times `margin`, plus
        `extra`, so that renders allocate nothing and never read back to the host."""
        n = self.g.n
        need = [0, 0]
        for slot, cams in ((0, self.ccams), (1, self.chalf if self.n_secondary else [])):
            fr = self.frames[slot]
            for cam in cams:
                self.ctx.render(self.g, cam, self.ro, fr)
                need[slot] = max(need[slot], fr.info()[0])
        self.pair_caps = [int(need[0] * margin) + extra, int(need[1] * margin) + extra]
        for slot, fr in enumerate(self.frames):
            cam = self.ccams[0] if slot == 0 else self.chalf[0]
            fr.reserve(n, cam.width, cam.height, self.pair_caps[min(slot, 1)])
        self.graphs = {}

    def check_status(self, margin=1.25):
        """gsn_sync_status: {counter: value} since the last check.  After a pair-capacity overflow the
        frames are reserved again with room for the largest view seen and captured sweeps are dropped."""
        from . import gsn as G
        st, stats, msg = self.ctx.sync_status()
        if st == G.GSN_E_CAPACITY:
            need = int(stats["pairs_needed"] * margin)
            self.pair_caps = [max(c, need) for c in self.pair_caps]
            for slot, fr in enumerate(self.frames):
                cam = self.ccams[0] if slot == 0 else self.chalf[0]
                fr.reserve(self.g.n, cam.width, cam.height, self.pair_caps[min(slot, 1)])
            for gr in getattr(self, "graphs", {}).values():
                gr.close()
            self.graphs = {}
        stats["status"] = st
        stats["message"] = msg
        return stats

    def sweep_graph(self, t, group_mask=31):
        """One jacobi sweep on image t as a replay of a captured HIP graph (captured on first use;
        needs reserve_frames).  Results equal sweep(t, group_mask)."""
        key = (int(t), int(group_mask))
        gr = self.graphs.get(key)
        if gr is None:
            gr = self.ctx.capture(lambda: self.sweep(t, group_mask))
            self.graphs[key] = gr
        gr.launch()

    def solve_opts(self, t):
        c = self.cams[t]
        return gsn.solve_opts(c.width * c.height, kappa=self.ro.kappa, **self.solve_kw)

    def accumulate(self, t):
        """Primary and secondary renders and block accumulation for training image t."""
        self.ctx.blocks_zero(self.blocks)
        cams = [self.ccams[t]] + [self.chalf[j] for j in self.knn[t]]
        tgts = [self.targets[t]] + [self.half_targets[j] for j in self.knn[t]]
        self.ctx.accumulate_views(self.g, cams, self.frames[:len(cams)], tgts, self.ro, self.lo, self.blocks,
                                  self.loss)

    def sweep(self, t, group_mask=31):
        """Jacobi schedule: every group linearised at the same state, one render and
        accumulation per view, the steps of the groups in group_mask applied together."""
        self.accumulate(t)
        self.ctx.solve_apply(self.g, self.ccams[t], self.blocks, self.solve_opts(t), self.steps, group_mask)

    def sweep_series(self, t, order=(1, 2, 4, 8, 16)):
        """Series schedule (Sec. 4.2, groups solved one after another: position, rotation,
        scaling, opacity, colour): for each group mask in `order`, render and accumulate the
        views at the state the previous groups left, solve, and apply that group only."""
        for m in order:
            self.sweep(t, m)

    # ------------------------------------------------------- first-order baseline
    def sweep_first_order(self, t, lr, adam=True, group_mask=31, beta1=0.9, beta2=0.999, eps=1e-15):
        """One first-order iteration on image t with the same gradients as a sweep (the blocks'
        gradient rows, summed over the primary and its secondaries): gradient descent or Adam
        with per-group learning rates (position, rotation, scaling, opacity, colour)."""
        if getattr(self, "fo_state", None) is None:
            K = (self.g.sh_degree + 1) ** 2
            self.fo_state = torch.zeros(2, 10 + 3 * K, max(self.g.n, 1), dtype=torch.float32, device=self.dev)
            self.fo_t = 0
        self.fo_t += 1
        self.accumulate(t)
        self.ctx.first_order_step(self.g, self.blocks, self.solve_opts(t), lr, adam=adam, step=self.fo_t,
                                  state=self.fo_state, beta1=beta1, beta2=beta2, eps=eps, group_mask=group_mask)

    # ------------------------------------------------------------ learned form
    def _accumulate_primary(self, t):
        self.ctx.blocks_zero(self.blocks)
        fr = self.frames[0]
        self.ctx.render(self.g, self.ccams[t], self.ro, fr)
        self.ctx.accumulate_hessian(self.g, fr, self.targets[t], self.lo, 0, self.blocks, self.loss[0])

    def _accumulate_held(self, t):
        """All views of image t accumulated with their shares of the summed rows left in the frames."""
        self.ctx.blocks_zero(self.blocks)
        cams = [self.ccams[t]] + [self.chalf[j] for j in self.knn[t]]
        tgts = [self.targets[t]] + [self.half_targets[j] for j in self.knn[t]]
        self.ctx.accumulate_views(self.g, cams, self.frames[:len(cams)], tgts, self.ro, self.lo, self.blocks,
                                  self.loss, add_shares=False)

    @staticmethod
    def _primary_only(so):
        """The solve options taking the primary's view slot alone (the secondaries' slots may be filled)."""
        sp = gsn.CSolveOpts.from_buffer_copy(so)
        sp.view_limit = 1
        return sp

    def _learned_buffers(self):
        n = self.g.n
        if getattr(self, "feat", None) is not None:
            return
        self.feat = torch.zeros(gsn.GSN_MLP_IN, max(n, 1), dtype=torch.float32, device=self.dev)
        # neighbouring-view residual of each kernel, cached from its last full-rule sweep (a feature)
        self.resid = torch.zeros(max(n, 1), dtype=torch.float32, device=self.dev)
        self.ok = torch.zeros(max(n, 1), dtype=torch.uint8, device=self.dev)
        self.alpha = torch.zeros(5, max(n, 1), dtype=torch.float32, device=self.dev)
        self.label = torch.zeros(5, max(n, 1), dtype=torch.float32, device=self.dev)
        self.mask = torch.zeros(5, max(n, 1), dtype=torch.float32, device=self.dev)
        self.steps_prim = gsn.Steps(n, self.g.sh_degree, self.dev)
        # over the full-rule sweeps: sum of |alpha_mlp - alpha_eff| and number of labelled entries
        self.err = torch.zeros(2, dtype=torch.float64, device=self.dev)

    def enable_learned(self, params, every=4, lr=1e-3, alpha_mode="mlp", alpha_const=1.0, mlp=None):
        """Learned form.  alpha_mode "mlp": the network's per-kernel scales; the controls "one" (the
        primary-only Newton step unscaled) and "const" (every kernel and group scaled by alpha_const)
        keep the same schedule of full-rule sweeps.  mlp: a network (gsn.MLP) to start from, e.g. one
        pre-trained on logged plain sweeps; else one from params."""
        self._learned_buffers()
        if mlp is None:
            mlp = gsn.MLP(params, self.dev)
            self.ctx.mlp_reset(mlp)
        self.mlp = mlp
        self.every = int(every)
        self.lr = float(lr)
        self.alpha_mode = alpha_mode
        self.alpha_const = float(alpha_const)
        self.mlp_loss = torch.zeros(1, dtype=torch.float64, device=self.dev)
        # kernels whose features left the trained range on the current sweep, and the counts of the
        # last learned sweeps on their way to the host (pinned words and the events that mark them)
        self.out_of_range = torch.zeros(1, dtype=torch.int32, device=self.dev)
        self._oor_words = [torch.zeros(1, dtype=torch.int32, pin_memory=True) for _ in range(3)]
        self._oor_pending = []
        self._oor_next = 0
        self.fallback_sweeps = 0

    def log_sweep(self, t, log, group_mask=31, max_rows=50000, seed=0):
        """A plain (full-rule) sweep on image t that also logs, for the learned form, the features of
        the primary-only blocks and the labels alpha_eff comparing the primary-only and full-rule
        steps: appends (features [17, m], labels [5, m], mask [5, m]) of at most max_rows labelled
        kernels (a seeded random subset) to `log`, then applies the full-rule step."""
        self._learned_buffers()
        so = self.solve_opts(t)
        n = self.g.n
        self._accumulate_held(t)
        self.ctx.add_view_shares(self.blocks, self.frames[:1])
        self.ctx.local_newton_solve(self.g, self.ccams[t], self.blocks, self._primary_only(so), self.steps_prim)
        self.ctx.step_features(self.g, self.ccams[t], self.blocks, so, self.feat[:, :n], self.ok[:n],
                               resid=self.resid[:n])
        self.ctx.add_view_shares(self.blocks, self.frames[1:1 + len(self.knn[t])])
        if self.n_secondary:
            self.ctx.neighbour_residual(self.blocks, self.resid[:n])
        self.ctx.local_newton_solve(self.g, self.ccams[t], self.blocks, so, self.steps)
        self.ctx.step_labels(self.steps_prim, self.steps, self.label[:, :n], self.mask[:, :n], ok=self.ok[:n])
        rows = torch.nonzero(self.mask[:, :n].amax(0) > 0).flatten()
        if rows.numel() > max_rows:
            gen = torch.Generator(device=self.dev).manual_seed(int(seed))
            rows = rows[torch.randperm(rows.numel(), generator=gen, device=self.dev)[:max_rows]]
        log.append((self.feat[:, rows].clone(), self.label[:, rows].clone(), self.mask[:, rows].clone()))
        self.ctx.apply_step(self.g, self.steps, so, group_mask)

    def sweep_learned(self, t, i, group_mask=31, check_range=True):
        """Sweep i of the learned form on training image t.  Every `every`-th sweep runs the full
        rule.  The overshoot rule is also the network's fallback: kernels whose features leave the
        trained range get no step on a learned sweep (alpha 0), and with check_range the learned sweep
        two after it runs the full rule (the count travels to the host without a wait: by then the
        device has long finished the sweep that counted it)."""
        so = self.solve_opts(t)
        n = self.g.n
        full = i % self.every == 0
        if check_range and len(self._oor_pending) >= 2:
            ev, word = self._oor_pending.pop(0)
            ev.synchronize()
            if int(word[0]) > 0 and not full:
                full = True
                self.fallback_sweeps += 1
        if full:
            # every view rendered and accumulated at once, the secondaries' shares of the summed rows
            # held back: the blocks then hold the primary's system, as after _accumulate_primary
            self._accumulate_held(t)
            self.ctx.add_view_shares(self.blocks, self.frames[:1])
            self.ctx.local_newton_solve(self.g, self.ccams[t], self.blocks, self._primary_only(so), self.steps_prim)
        else:
            self._accumulate_primary(t)
            self.ctx.local_newton_solve(self.g, self.ccams[t], self.blocks, so, self.steps)
        self.ctx.step_features(self.g, self.ccams[t], self.blocks, so, self.feat[:, :n], self.ok[:n],
                               resid=self.resid[:n])
        self.out_of_range.zero_()
        self.ctx.mlp_infer(self.mlp, self.feat[:, :n], self.ok[:n], self.alpha[:, :n], self.out_of_range)
        if check_range and not full:
            word = self._oor_words[self._oor_next]
            self._oor_next = (self._oor_next + 1) % len(self._oor_words)
            word.copy_(self.out_of_range, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record()
            self._oor_pending.append((ev, word))
        if not full:
            if self.alpha_mode == "one":
                self.ctx.apply_step(self.g, self.steps, so, group_mask)
            else:
                if self.alpha_mode == "const":
                    self.alpha.fill_(self.alpha_const)
                self.ctx.apply_step(self.g, self.steps, so, group_mask, scale=self.alpha[:, :n])
            return
        # full rule: the secondaries' blocks join the primary's; label and train, then apply the full step
        self.ctx.add_view_shares(self.blocks, self.frames[1:1 + len(self.knn[t])])
        if self.n_secondary:
            self.ctx.neighbour_residual(self.blocks, self.resid[:n])
        # the full step applied with its solve (the labels and the training read the steps only)
        self.ctx.solve_apply(self.g, self.ccams[t], self.blocks, so, self.steps, group_mask)
        self.ctx.step_labels(self.steps_prim, self.steps, self.label[:, :n], self.mask[:, :n], ok=self.ok[:n],
                             alpha=self.alpha[:, :n], err=self.err)
        self.ctx.mlp_train_step(self.mlp, self.feat[:, :n], self.label[:, :n], self.mask[:, :n], lr=self.lr,
                                loss=self.mlp_loss)


    def learned_error(self):
        """Mean |alpha_mlp - alpha_eff| over the labelled entries of the full-rule sweeps so far."""
        e = self.err.cpu().numpy()
        if e[1] <= 0:
            return None
        return float(e[0] / e[1])

    def close(self):
        for f in self.frames:
            f.close()
        self.ctx.close()


def pretrain(ctx, mlp, logs, epochs=5, batch=8192, lr=1e-2, seed=0):
    """Trains the step-scale network on logged plain sweeps (log_sweep): Adam steps of the library
    on shuffled mini-batches of the logged (features, labels, mask) rows.  Returns the mean loss
    of each epoch."""
    F = torch.cat([x[0] for x in logs], 1)
    Lb = torch.cat([x[1] for x in logs], 1)
    M = torch.cat([x[2] for x in logs], 1)
    m = F.shape[1]
    gen = torch.Generator(device=F.device).manual_seed(int(seed))
    loss = torch.zeros(1, dtype=torch.float64, device=F.device)
    curve = []
    for _ in range(epochs):
        perm = torch.randperm(m, generator=gen, device=F.device)
        tot = torch.zeros(1, dtype=torch.float64, device=F.device)
        nb = 0
        for b0 in range(0, m, batch):
            idx = perm[b0:b0 + batch]
            ctx.mlp_train_step(mlp, F[:, idx].contiguous(), Lb[:, idx].contiguous(), M[:, idx].contiguous(), lr=lr,
                               loss=loss)
            tot += loss
            nb += 1
        curve.append(float((tot / max(nb, 1)).cpu()))
    return curve
