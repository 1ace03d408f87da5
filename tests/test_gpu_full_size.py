"""GPU parity at the benchmark's full size: 1M Gaussians at SH degree 3 on one 1920x1080 view,
rendered and accumulated by the same library calls and launch shapes the benchmark times (its
pair lists take the large-sort path).  The per-tile lists are compared bit-exactly over the
whole frame, the image, transmittance, loss value and loss maps element by element, and the
blocks of sampled kernels against the oracle's blocks of the same kernels (the oracle computes
them one kernel at a time).

A frame this size has a few hundred pixels whose threshold decisions sit within rounding of a
threshold (single- and double-precision compositing may decide them differently, by up to a
whole splat's colour).  The SSIM window couples every pixel's loss derivatives to the pixels
within 10 of it (a window of radius 5 around each window centre of radius 5), so the loss maps
are compared away from those pixels, and the blocks of kernels that any such pixel composited
are not compared."""
import numpy as np
import pytest

from oracle import oracle as O
from synth.scenes import make_config
from tests.parity import (BLOCK_GROUPS, TOL_GRAD, TOL_IMAGE, blocks_gpu_to_oracle_view, compare_binning, gpu_view,
                          kernels_in_reach, near_threshold_kernels, pixel_mask, rel_inf, ssim_reach)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# The mixed form's bars at this size.  Its SSIM window sums in single precision lose to the
# variance's cancellation (E[u^2] - mu^2 over an 11x11 window) in flat regions: measured dL 1.7e-5 and
# h 7.6e-5 of their largest values on the 1080p view (1.2e-5 and 4.4e-5 on the 540p one), so the maps'
# bar is 1e-4.  The blocks, sums of single-precision pair terms over up to ~10^4 pixels per kernel,
# measure at most 8.8e-6: bar 2e-5.
MIXED_FULL_TOL_MAPS = 1e-4
MIXED_FULL_TOL_BLOCKS = 2e-5


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


def _full_size_view(gsn, ctx, g, cam, tgt, tiles, label, gpu_cam=None):
    """gpu_cam: the library's camera for the view (default: the same camera as the oracle's)."""
    lam = 0.2
    dg = gsn.DeviceGaussians.from_host(g)
    blocks = gsn.Blocks(g.n, 1, ctx.device)
    ctx.blocks_zero(blocks)
    gv = gpu_view(ctx, gsn, dg, cam if gpu_cam is None else gpu_cam, torch.tensor(tgt, device=ctx.device), lam,
                  blocks, 0, keep=False)
    fr = O.render(g, cam, O.opts(lambda_ssim=lam), g32=g)
    ov = {"fr": fr}
    # lists: bit-exact on every tile of the frame
    assert compare_binning(gv, ov, g.n) == tiles
    assert gv["pairs"] > 1 << 22  # more pairs than the small-sort threshold
    # image and compositing decisions
    mask = pixel_mask(ov)
    assert (~mask).sum() < 1e-3 * mask.size
    assert rel_inf(gv["img"][:, mask], fr.img[:, mask]) < TOL_IMAGE
    assert rel_inf(gv["T"][mask], fr.Tfinal[mask]) < TOL_IMAGE
    assert np.array_equal(gv["ncontrib"][mask], fr.ncontrib[mask])
    # loss and its per-pixel derivative maps, away from the ambiguous pixels' SSIM reach
    parts, dL, hd = O.loss(fr.img, tgt, lam)
    assert abs(gv["loss"][0] - parts[0]) < TOL_GRAD * abs(parts[0])
    assert abs(gv["loss"][1] - parts[1]) < TOL_GRAD * abs(parts[1])
    reach = ssim_reach(mask)
    far = ~reach
    assert far.sum() > 0.8 * far.size
    assert rel_inf(gv["dL"][:, far], dL[:, far]) < TOL_GRAD
    assert rel_inf(gv["h"][:, far], hd[:, far]) < TOL_GRAD
    # blocks of sampled kernels, none composited at a pixel within that reach (per tile: the list
    # prefix up to the longest such pixel's last composited entry).  Most of the million kernels
    # are hidden behind others, so the sample is drawn from the kernels in the front of some
    # tile's list (the prefix that the tile's median pixel composites or passes): the 32 in the
    # most such fronts (they set each group's scale) and 368 of the others at random.  Those the
    # oracle finds composited nowhere must have all-zero blocks on the GPU too.
    keep = fr.vis.astype(bool) & ~near_threshold_kernels(fr, g.n) & ~kernels_in_reach(fr, reach, g.n)
    assert keep.sum() > 0.5 * g.n
    tx = (cam.width + 15) // 16
    front = np.zeros(g.n, np.int64)
    for t in range(len(fr.tile_start) - 1):
        ty, tx0 = divmod(t, tx)
        m = int(np.median(fr.ncontrib[16 * ty:16 * ty + 16, 16 * tx0:16 * tx0 + 16]))
        front[fr.ids[fr.tile_start[t]:fr.tile_start[t] + m]] += 1
    front[~keep] = 0
    big = np.argsort(front)[-32:]
    rest = np.setdiff1d(np.nonzero(front > 0)[0], big)
    sel = np.sort(np.concatenate([big, np.random.default_rng(5).choice(rest, 368, replace=False)]))
    want = O.blocks(g, fr, dL, hd, sel)
    got = blocks_gpu_to_oracle_view(blocks.view()[:, torch.as_tensor(sel, device=ctx.device)].cpu().numpy(), 0)
    covered = want[:, 38] > 0
    assert covered.sum() >= 100
    assert np.all(got[~covered] == 0.0)
    got, want = got[covered], want[covered]
    errs = {name: rel_inf(got[:, sl], want[:, sl]) for name, sl in BLOCK_GROUPS.items()}
    print(f"\n[{label}] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for name, e in errs.items():
        assert e < TOL_GRAD, (name, e)
    # the mixed precision form (single-precision SSIM sums, statistic sums and rotation/scale chain) on
    # the same view, against the same oracle values
    mb = gsn.Blocks(g.n, 1, ctx.device)
    ctx.blocks_zero(mb)
    mv = gpu_view(ctx, gsn, dg, cam if gpu_cam is None else gpu_cam, torch.tensor(tgt, device=ctx.device), lam,
                  mb, 0, keep=False, precision=1)
    merrs = {"dL": rel_inf(mv["dL"][:, far], dL[:, far]), "h": rel_inf(mv["h"][:, far], hd[:, far]),
             "loss_S": abs(mv["loss"][1] - parts[1]) / abs(parts[1])}
    mgot = blocks_gpu_to_oracle_view(mb.view()[:, torch.as_tensor(sel, device=ctx.device)].cpu().numpy(), 0)
    assert np.all(mgot[~covered] == 0.0)
    mgot = mgot[covered]
    merrs.update({name: rel_inf(mgot[:, sl], want[:, sl]) for name, sl in BLOCK_GROUPS.items()})
    print(f"[{label}, mixed form] " + " ".join(f"{k}={v:.2e}" for k, v in merrs.items()), flush=True)
    for name, e in merrs.items():
        assert e < (MIXED_FULL_TOL_MAPS if name in ("dL", "h") else MIXED_FULL_TOL_BLOCKS), (name, e)


@pytest.fixture(scope="module")
def scene():
    cfg = make_config("c2")
    assert (cfg.init.n, cfg.cams[0].width, cfg.cams[0].height) == (1_000_000, 1920, 1080)
    return cfg


def test_full_size_view_parity(gsn, ctx, scene):
    """The primary view: 1920x1080, 120 x 68 tiles."""
    cam = scene.cams[0]
    tgt = O.render(scene.gt, cam, O.opts()).img.astype(np.float32)
    _full_size_view(gsn, ctx, scene.init, cam, tgt, 120 * 68, "full-size")


def test_full_size_secondary_view_parity(gsn, ctx, scene):
    """A half-resolution secondary view (960x540, 60 x 34 tiles, the last tile row ragged) with its
    target the 2x2 box downsampling of the full-resolution one, as the sweep forms it."""
    cam = scene.cams[1]
    tgt = O.downsample(O.render(scene.gt, cam, O.opts()).img.astype(np.float32)).astype(np.float32)
    _full_size_view(gsn, ctx, scene.init, O.half_camera(cam), tgt, 60 * 34, "full-size secondary",
                    gpu_cam=gsn.camera_half(gsn.camera(cam)))
