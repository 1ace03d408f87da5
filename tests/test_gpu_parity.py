"""GPU parity: the HIP library (called through its C ABI) against the FP64 oracle.

Bars: tile keys, rectangles and per-tile lists bit-exact; images, loss maps,
gradients and Hessian blocks within 1e-5 (relative infinity norm per tensor
and per attribute group); Newton steps within 1e-4 per group.  Pixels whose
oracle threshold decisions lie within 1e-5 (relative) of a threshold are not
compared element-wise, nor the kernels composited there (single- and
double-precision compositing may take those decisions differently); their
count is reported.  Loss maps are compared, and kernels kept, only beyond the
SSIM windows' 10-pixel reach of such pixels.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_config
from tests.parity import (BLOCK_GROUPS, STEP_GROUPS, TOL_GRAD, TOL_IMAGE, TOL_STEP, blocks_gpu_to_oracle_view,
                          compare_binning, gpu_view, near_threshold_kernels, oracle_frames, oracle_view,
                          summed_to_gpu_blocks, rel_inf,
                          step_sensitivity, view_errors, zstats_gpu_to_full, zstats_to_frame)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_13975_amd import gsn as G
    return G


@pytest.fixture(scope="module")
def ctx(gsn):
    c = gsn.Context(0)
    yield c
    c.close()


def _report(name, errs):
    print(f"\n[{name}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)


def _check_view(gsn, ctx, g, cam, tgt, lam, label, gn=False):
    dg = gsn.DeviceGaussians.from_host(g)
    blocks = gsn.Blocks(g.n, 1, ctx.device)
    ctx.blocks_zero(blocks)
    gv = gpu_view(ctx, gsn, dg, cam, torch.tensor(tgt, device=ctx.device), lam, blocks, 0, gn=gn)
    ov = oracle_view(g, cam, tgt, lam, gn=gn)
    ntiles = compare_binning(gv, ov, g.n)
    blk = blocks.view().cpu().numpy()
    errs, keep = view_errors(g, cam, gv, ov, blk)
    errs = {"tiles": ntiles, "pairs": gv["pairs"], **errs}
    fr = ov["fr"]
    _report(label, errs)
    dump = os.environ.get("GSN_DUMP_DIR")
    if dump:
        os.makedirs(dump, exist_ok=True)
        np.savez_compressed(os.path.join(dump, f"view_{label}.npz"), gpu_z=gv["z"], gpu_rec=gv["rec"], orc_z=ov["z"],
                            gpu_blocks=blk, orc_blocks=ov["blocks"], gpu_img=gv["img"], gpu_dL=gv["dL"],
                            gpu_h=gv["h"], orc_img=fr.img, orc_dL=ov["dL"], orc_h=ov["hd"])
    assert errs["img"] < TOL_IMAGE and errs["T"] < TOL_IMAGE
    assert errs["ncontrib_mismatch"] == 0
    assert errs["loss_L2"] < TOL_GRAD and errs["loss_S"] < TOL_GRAD
    assert errs["dL"] < TOL_GRAD and errs["h"] < TOL_GRAD
    assert errs["z_g"] < TOL_GRAD and errs["z_H"] < TOL_GRAD and errs["z_w"] < TOL_GRAD
    for name in BLOCK_GROUPS:
        assert errs[name] < TOL_GRAD, (name, errs[name])
    return dg, blocks, gv, ov, keep


def test_c0_view_parity(gsn, ctx):
    """256 kernels, 64x64, SH degree 0 (the oracle-scale workload)."""
    cfg = make_config("c0")
    cam = cfg.cams[0]
    tgt = O.render(cfg.gt, cam, O.opts()).img.astype(np.float32)
    _check_view(gsn, ctx, cfg.init, cam, tgt, 0.2, "c0")


def test_surface_scene_ragged_view_parity(gsn, ctx):
    """SH degree 3, anisotropic kernels, ragged tiles (250 x 190 is not a multiple of 16)."""
    cfg = make_config("c1", n=6000, width=250, height=190, n_views=6)
    cam = cfg.cams[2]
    tgt = O.render(cfg.gt, cam, O.opts()).img.astype(np.float32)
    _check_view(gsn, ctx, cfg.init, cam, tgt, 0.2, "c1-small")


def test_gauss_newton_view_parity(gsn, ctx):
    """Local Gauss-Newton statistics and blocks (no loss-gradient x image-curvature terms)."""
    cfg = make_config("c1", n=6000, width=250, height=190, n_views=6)
    cam = cfg.cams[2]
    tgt = O.render(cfg.gt, cam, O.opts()).img.astype(np.float32)
    _check_view(gsn, ctx, cfg.init, cam, tgt, 0.2, "c1-small gauss-newton", gn=True)


def test_deep_tile_list_parity(gsn, ctx):
    """One 16x16 tile with a 4000-entry list of faint kernels: pixels composite far past the
    batches whose composited pairs the forward pass records, so the backward pass evaluates
    the later batches itself and stages their pairs over several LDS rounds.  The target is the
    ground truth's render at half brightness: every pixel averages thousands of kernels, so a
    perturbed state renders within a few percent of its own ground truth, and the loss gradient
    (proportional to that residual) would carry the image's single-precision rounding amplified
    by the image-to-residual ratio (about 30 here) rather than the backward pass's own error."""
    from synth.scenes import deep_list_scene
    gt, g, cam = deep_list_scene(77)
    fr = O.render(gt, cam, O.opts())
    assert np.diff(fr.tile_start)[0] == 4000
    tgt = (0.5 * fr.img).astype(np.float32)
    ctx.profile_enable(True)
    _check_view(gsn, ctx, g, cam, tgt, 0.2, "deep-list")
    _, counts = ctx.profile_read()
    ctx.profile_enable(False)
    assert counts["bwd_evals"] > 0  # the evaluation path past the recorded batches ran


@pytest.mark.parametrize("lam,nsec,gn", [(0.0, 3, False), (0.2, 3, False), (0.2, 0, False), (0.2, 8, False),
                                         (0.2, 3, True)])
def test_sweep_steps_parity(gsn, ctx, lam, nsec, gn):
    """Primary + K half-resolution KNN secondaries (|N_t| in {0, 3, 8}), solve and apply (Sec.
    4.2-4.3); gn: the local Gauss-Newton blocks."""
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=10)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    g = cfg.init
    t = 3
    V = nsec + 1
    knn_o = O.camera_knn(cfg.cams, g, nsec) if nsec else None
    # end to end with the colour trust radius open (the radius itself is checked on the solve stage below)
    o = O.opts(lambda_ssim=lam, trust_sh=1e30, gauss_newton=int(gn))
    res = O.sweep(g, cfg.cams, tg, t, knn_o, o)
    # kernels that any view composites at a pixel with a near-threshold decision are not compared
    bad = np.zeros(g.n, bool)
    for fr in res["frames"]:
        bad |= near_threshold_kernels(fr, g.n)
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    dg = gsn.DeviceGaussians.from_host(g)
    tr = LocalNewtonTrainer(dg, cfg.cams, [torch.tensor(x, device=ctx.device) for x in tg], nsec, lam,
                            solve_kw={"trust_sh": 1e30}, gauss_newton=gn)
    assert tr.blocks.n_views == V
    if nsec:  # the library's scene centre and KNN table (Sec. 4.1) against the oracle's
        assert np.array_equal(knn_o, tr.knn)
    tr.accumulate(t)
    so = tr.solve_opts(t)
    tr.ctx.local_newton_solve(tr.g, tr.ccams[t], tr.blocks, so, tr.steps)
    st, fl = (x.cpu().numpy() for x in tr.steps.view())
    torch.cuda.synchronize()
    errs = {}
    dec_o = res["dec"]
    agree = np.all(fl[:4].T == dec_o[:, :4], axis=1)
    vis = dec_o[:, 0] != -2
    errs["visible"] = int(vis.sum())
    errs["decision_agreement"] = float(agree[vis].mean())
    errs["excluded_near_threshold"] = int((bad & vis).sum())
    keep = agree & vis & ~bad
    K = (g.sh_degree + 1) ** 2
    o_same = res["opts"]
    gb = tr.blocks.view().cpu().numpy()
    # (1) end to end, where the step is determined at the blocks' precision (1e-5)
    sens = step_sensitivity(g, cfg.cams[t], o_same, res["summed"], V)
    groups = list(STEP_GROUPS.items()) + [("colour", slice(11, 11 + 3 * K))]
    for i, (name, sl) in enumerate(groups):
        ok = keep & (sens[:, i] <= 1e-5)
        errs["determined_" + name] = int(ok.sum())
        errs[name] = rel_inf(st[sl].T[ok], res["steps"][ok, sl])
    # (2) the solve stage alone: the oracle's blocks, rounded to the library's float32 storage,
    # solved by the library and by the oracle
    S32 = res["summed"].astype(np.float32).astype(np.float64)
    tr.blocks.view().copy_(torch.tensor(summed_to_gpu_blocks(S32, V), dtype=torch.float32, device=ctx.device))
    tr.ctx.local_newton_solve(tr.g, tr.ccams[t], tr.blocks, so, tr.steps)
    st_s, fl_s = (x.cpu().numpy() for x in tr.steps.view())
    want_s, dec_s = O.solve(g, cfg.cams[t], o_same, S32, V)
    same = np.all(fl_s[:4].T == dec_s[:, :4], axis=1) & vis
    errs["solver_decisions"] = float(same[vis].mean())
    for name, sl in groups:
        errs["solver_" + name] = rel_inf(st_s[sl].T[same], want_s[same, sl])
    # the overlap numerator row end to end (the sum over the views of sum (alpha T)^2)
    errs["overlap_row"] = rel_inf(gb[30 + 10 * V][keep], res["summed"][keep, 39 + 10 * V])
    # the same with a step fraction, with the default colour trust radius and with the overlap share
    for tag, field, ofield, val in (("frac", "step_frac", "step_frac", 0.3), ("trust", "trust_sh", "trust_sh", 1.0),
                                    ("overlap", "overlap_scale", "overlap", 1)):
        so_f = tr.solve_opts(t)
        setattr(so_f, field, val)
        tr.ctx.local_newton_solve(tr.g, tr.ccams[t], tr.blocks, so_f, tr.steps)
        st_f, fl_f = (x.cpu().numpy() for x in tr.steps.view())
        o_f = o_same.copy()
        o_f[O.O_NAMES.index(ofield)] = val
        want_f, dec_f = O.solve(g, cfg.cams[t], o_f, S32, V)
        same_f = np.all(fl_f[:4].T == dec_f[:, :4], axis=1) & vis
        for name, sl in groups:
            errs[f"solver_{tag}_" + name] = rel_inf(st_f[sl].T[same_f], want_f[same_f, sl])
    dump = os.environ.get("GSN_DUMP_DIR")
    if dump:
        os.makedirs(dump, exist_ok=True)
        np.savez_compressed(os.path.join(dump, f"sweep_lam{lam}_N{nsec}_gn{int(gn)}.npz"), gpu_blocks=gb,
                            gpu_steps=st, gpu_flags=fl,
                            orc_summed=res["summed"], orc_steps=res["steps"], orc_dec=res["dec"], bad=bad,
                            sens=sens)
    _report(f"sweep-steps lam={lam} |N_t|={nsec} gn={gn}", errs)
    assert errs["decision_agreement"] > 0.99 and errs["solver_decisions"] > 0.999
    # kernels composited at a pixel whose threshold decision is ambiguous are left out of the end-to-end
    # comparison (17% of the visible ones in this scene with three secondaries; none without): a ceiling
    # keeps that share from growing unnoticed
    assert errs["excluded_near_threshold"] <= 0.2 * errs["visible"], errs["excluded_near_threshold"]
    assert errs["overlap_row"] < TOL_GRAD
    for name, _ in groups:
        assert errs["solver_" + name] < 1e-5, ("solver", name, errs["solver_" + name])
        assert errs["solver_frac_" + name] < 1e-5, ("solver, step fraction", name, errs["solver_frac_" + name])
        assert errs["solver_trust_" + name] < 1e-5, ("solver, colour radius", name, errs["solver_trust_" + name])
        # scaled by the overlap share the largest steps are rarely trust-clamped, so the relative measure is
        # set by ill-conditioned unclamped steps: the Newton-step bar (1e-4) applies
        assert errs["solver_overlap_" + name] < TOL_STEP, ("solver, overlap share", name,
                                                         errs["solver_overlap_" + name])
        assert errs[name] < TOL_STEP, (name, errs[name])
        assert errs["determined_" + name] > 0.5 * errs["visible"], ("too few determined steps", name)
    # (3) apply: the oracle's steps (float32, as the library stores them) applied by both sides
    st32 = want_s.astype(np.float32)
    sv, fv = tr.steps.view()
    sv.copy_(torch.tensor(st32.T, device=ctx.device))
    fv[:4].copy_(torch.tensor(dec_s[:, :4].T.astype(np.int32), device=ctx.device))
    fv[4].copy_(torch.tensor(dec_s[:, 4].astype(np.int32), device=ctx.device))
    tr.ctx.apply_step(tr.g, tr.steps, so, 31)
    new_g = tr.g.to_host()
    new_o = O.apply(g, st32.astype(np.float64), dec_s, o, 31)
    for a in ("pos", "rot", "scale", "opac", "sh"):
        assert np.allclose(getattr(new_g, a), getattr(new_o, a), rtol=2e-6, atol=2e-6), a
    tr.close()


def test_series_stages_parity(gsn, ctx):
    """Series schedule (Sec. 4.2: position, rotation, scaling, opacity, colour, each group
    linearised at the state the previous groups left).  Every stage of the library's
    sweep_series starts from the oracle's state after the previous stage, rounded to float32,
    and its applied change of that group matches the oracle's stage on the kernels whose step
    is determined at the blocks' precision."""
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    from synth.scenes import Gaussians
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=10)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    tg_d = [torch.tensor(x, device=ctx.device) for x in tg]
    t, K, V = 3, 3, 4
    knn = O.camera_knn(cfg.cams, cfg.init, K)
    o = O.opts(lambda_ssim=0.2, trust_sh=1e30, step_frac=0.5)
    state = cfg.init
    attr = {1: "pos", 2: "rot", 4: "scale", 8: "opac", 16: "sh"}
    errs = {}
    for gi, m in enumerate((1, 2, 4, 8, 16)):
        g32 = Gaussians(*(np.asarray(getattr(state, a), np.float32) for a in ("pos", "rot", "scale", "opac", "sh")),
                        cfg.init.sh_degree)
        new_o, stages = O.sweep_series(g32, cfg.cams, tg, t, knn, o, (m,))
        res = stages[0]
        dg = gsn.DeviceGaussians.from_host(g32)
        tr = LocalNewtonTrainer(dg, cfg.cams, tg_d, K, 0.2, solve_kw={"trust_sh": 1e30, "step_frac": 0.5})
        tr.sweep_series(t, (m,))
        new_g = dg.to_host()
        fl = tr.steps.view()[1].cpu().numpy()
        tr.close()
        vis = res["dec"][:, 0] != -2
        agree = np.all(fl[:4].T == res["dec"][:, :4], axis=1)
        bad = np.zeros(g32.n, bool)
        for fr in res["frames"]:
            bad |= near_threshold_kernels(fr, g32.n)
        sens = step_sensitivity(g32, cfg.cams[t], res["opts"], res["summed"], V)
        keep = vis & agree & ~bad & (sens[:, gi] <= 1e-5)
        a = attr[m]
        base = np.asarray(getattr(g32, a), np.float64)
        dg_ = (np.asarray(getattr(new_g, a), np.float64) - base)[..., keep]
        do_ = (np.asarray(getattr(new_o, a), np.float64) - base)[..., keep]
        errs[f"{a}_kept"] = int(keep.sum())
        errs[a] = rel_inf(dg_, do_)
        # the other groups are left alone by this stage
        for b in attr.values():
            if b != a:
                assert np.array_equal(np.asarray(getattr(new_g, b)), np.asarray(getattr(g32, b))), (a, b)
        # after the geometry stages many kernels are composited at near-threshold pixels
        assert keep.sum() > 0.25 * vis.sum(), (a, int(keep.sum()), int(vis.sum()))
        state = new_o
    _report("series stages", errs)
    for a in attr.values():
        assert errs[a] < TOL_STEP, (a, errs[a])


def test_c0_sweeps_lower_the_loss_like_the_oracle(gsn, ctx):
    """Five sweeps on the 256-kernel scene at step fraction 0.3: the library's loss before each
    sweep follows the oracle's run from the same start (each side carries its own state)."""
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    cfg = make_config("c0")
    cam = cfg.cams[0]
    tgt = O.render(cfg.gt, cam, O.opts()).img.astype(np.float32)
    g, want = cfg.init, []
    for _ in range(5):
        res = O.sweep(g, cfg.cams, [tgt], 0, None, O.opts(step_frac=0.3))
        want.append(res["losses"][0][0] + 0.2 * res["losses"][0][1])
        g = res["new"]
    dg = gsn.DeviceGaussians.from_host(cfg.init)
    tr = LocalNewtonTrainer(dg, cfg.cams, [torch.tensor(tgt, device=ctx.device)], 0, 0.2,
                            solve_kw={"step_frac": 0.3})
    got = []
    for _ in range(5):
        tr.sweep(0)
        lv = tr.loss[0].cpu().numpy()
        got.append(lv[0] + 0.2 * lv[1])
    tr.close()
    _report("c0 sweeps", {f"loss{i}": v for i, v in enumerate(got)})
    assert all(b < a for a, b in zip(got, got[1:])), got
    assert np.allclose(got, want, rtol=1e-3, atol=0), (got, want)


def test_edge_cases(gsn, ctx):
    """No kernels; every kernel behind the camera; a single kernel."""
    cfg = make_config("c0")
    cam = cfg.cams[0]
    fr = ctx.frame()
    ro = gsn.render_opts()
    for n in (0, 1):
        g = cfg.init.subset(np.arange(n))
        dg = gsn.DeviceGaussians.from_host(g)
        rgb = torch.ones(3, cam.height, cam.width, device=ctx.device)
        ctx.render(dg, gsn.camera(cam), ro, fr, rgb)
        blocks = gsn.Blocks(n, 1, ctx.device)
        ctx.blocks_zero(blocks)
        tgt = torch.zeros(3, cam.height, cam.width, device=ctx.device)
        ctx.accumulate_hessian(dg, fr, tgt, gsn.loss_opts(), 0, blocks)
        torch.cuda.synchronize()
        want = O.render(g, cam, O.opts()).img if n else np.zeros((3, cam.height, cam.width))
        assert rel_inf(rgb.cpu().numpy(), want) < TOL_IMAGE or np.max(np.abs(want)) == 0
    g = cfg.init.copy()
    g.pos[2] -= 10.0  # all behind the camera
    dg = gsn.DeviceGaussians.from_host(g)
    rgb = torch.ones(3, cam.height, cam.width, device=ctx.device)
    ctx.render(dg, gsn.camera(cam), ro, fr, rgb)
    torch.cuda.synchronize()
    assert fr.info()[0] == 0 and float(rgb.abs().max()) == 0.0
    # invalid arguments are rejected before any launch
    with pytest.raises(gsn.GsnError):
        ctx.render(dg, gsn.camera(cam), gsn.CRenderOpts(8, 0.0039, 0.99, 1e-4, 0.3, 3.0), fr)
    fr.close()
