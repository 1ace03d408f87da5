"""GPU parity: the HIP library (called through its C ABI) against the FP64 oracle.

Bars: tile keys, rectangles and per-tile lists bit-exact; images, loss maps,
gradients and Hessian blocks within 1e-5 (relative infinity norm per tensor
and per attribute group); Newton steps within 1e-4 per group.  Pixels whose
oracle threshold decisions lie within 1e-4 (relative) of a threshold are not
compared element-wise (single- and double-precision compositing may take
those decisions differently); their count is reported.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_config
from tests.parity import (BLOCK_GROUPS, STEP_GROUPS, TOL_GRAD, TOL_IMAGE, TOL_STEP, blocks_gpu_to_oracle_view,
                          compare_binning, gpu_view, oracle_view, pixel_mask, rel_inf, zstats_gpu_to_full)

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


def _check_view(gsn, ctx, g, cam, tgt, lam, label):
    dg = gsn.DeviceGaussians.from_host(g)
    blocks = gsn.Blocks(g.n, 1, ctx.device)
    ctx.blocks_zero(blocks)
    gv = gpu_view(ctx, gsn, dg, cam, torch.tensor(tgt, device=ctx.device), lam, blocks, 0)
    ov = oracle_view(g, cam, tgt, lam)
    ntiles = compare_binning(gv, ov, g.n)
    mask = pixel_mask(ov)
    errs = {"tiles": ntiles, "pairs": gv["pairs"], "ambiguous_px": int((~mask).sum())}
    fr = ov["fr"]
    errs["img"] = rel_inf(gv["img"][:, mask], fr.img[:, mask])
    errs["T"] = rel_inf(gv["T"][mask], fr.Tfinal[mask])
    errs["ncontrib_mismatch"] = int((gv["ncontrib"][mask] != fr.ncontrib[mask]).sum())
    errs["loss_L2"] = abs(gv["loss"][0] - ov["parts"][0]) / abs(ov["parts"][0])
    errs["loss_S"] = abs(gv["loss"][1] - ov["parts"][1]) / abs(ov["parts"][1])
    errs["dL"] = rel_inf(gv["dL"][:, mask], ov["dL"][:, mask])
    errs["h"] = rel_inf(gv["h"][:, mask], ov["hd"][:, mask])
    # kernels that touch an ambiguous pixel are excluded from the per-kernel comparisons
    bad = np.zeros(g.n, bool)
    if (~mask).any():
        tx = (cam.width + 15) // 16
        ys, xs = np.nonzero(~mask)
        for y, x in zip(ys, xs):
            t = (y // 16) * tx + x // 16
            bad[fr.ids[fr.tile_start[t]:fr.tile_start[t + 1]]] = True
    keep = ~bad
    gz, Hz, wz = zstats_gpu_to_full(gv["z"])
    Zo = ov["z"]
    errs["z_g"] = rel_inf(gz[keep], Zo[keep, :9])
    errs["z_H"] = rel_inf(Hz[keep].reshape(-1, 81), Zo[keep, 9:90])
    errs["z_w"] = rel_inf(wz[keep], Zo[keep, 90])
    blk = blocks.view().cpu().numpy()
    Bg = blocks_gpu_to_oracle_view(blk, 0)
    for name, sl in BLOCK_GROUPS.items():
        errs[name] = rel_inf(Bg[keep][:, sl], ov["blocks"][keep][:, sl])
    _report(label, errs)
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


@pytest.mark.parametrize("lam", [0.0, 0.2])
def test_sweep_steps_parity(gsn, ctx, lam):
    """Primary + 3 half-resolution KNN secondaries, solve and apply (Sec. 4.2-4.3)."""
    cfg = make_config("c1", n=4000, width=200, height=150, n_views=8)
    tg = [O.render(cfg.gt, c, O.opts()).img.astype(np.float32) for c in cfg.cams]
    g = cfg.init
    t = 3
    knn_o = O.camera_knn(cfg.cams, g, 3)
    knn_g = gsn.camera_knn(np.stack([c.center for c in cfg.cams]),
                           np.asarray(g.pos, np.float64).mean(1), 3)
    assert np.array_equal(knn_o, knn_g)
    o = O.opts(lambda_ssim=lam)
    res = O.sweep(g, cfg.cams, tg, t, knn_o, o)
    from paper_2501_13975_amd.train import LocalNewtonTrainer
    dg = gsn.DeviceGaussians.from_host(g)
    tr = LocalNewtonTrainer(dg, cfg.cams, [torch.tensor(x, device=ctx.device) for x in tg], 3, lam)
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
    keep = agree & vis
    for name, sl in STEP_GROUPS.items():
        errs[name] = rel_inf(st[sl].T[keep], res["steps"][keep, sl])
    K = (g.sh_degree + 1) ** 2
    errs["colour"] = rel_inf(st[11:11 + 3 * K].T[keep], res["steps"][keep, 11:])
    _report(f"sweep-steps lam={lam}", errs)
    assert errs["decision_agreement"] > 0.99
    for name in list(STEP_GROUPS) + ["colour"]:
        assert errs[name] < TOL_STEP, (name, errs[name])
    # apply: the GPU update of the GPU steps equals the oracle update of the same steps
    tr.ctx.apply_step(tr.g, tr.steps, so, 31)
    new_g = tr.g.to_host()
    st64 = st.T.astype(np.float64)
    dec64 = fl.T.astype(np.int32)
    new_o = O.apply(g, st64, dec64, o, 31)
    for a in ("pos", "rot", "scale", "opac", "sh"):
        assert np.allclose(getattr(new_g, a), getattr(new_o, a), rtol=2e-6, atol=2e-6), a
    tr.close()


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
