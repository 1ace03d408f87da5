"""Shared helpers of the GPU parity tests: run one view through the HIP library
(C ABI via the ctypes binding) and through the FP64 oracle, and compare."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

# Tolerances (relative infinity norm per tensor / per attribute group).
TOL_IMAGE = 1e-5
TOL_GRAD = 1e-5
TOL_STEP = 1e-4
MARGIN = 1e-4  # oracle pixels whose threshold decisions sit this close to a threshold are not compared


def rel_inf(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = float(np.max(np.abs(b))) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


def sym_from_packed(p, n):
    """Packed upper triangle (row by row) [np, K] -> full [K, n, n]."""
    K = p.shape[1]
    H = np.zeros((K, n, n))
    idx = 0
    for i in range(n):
        for j in range(i, n):
            H[:, i, j] = p[idx]
            H[:, j, i] = p[idx]
            idx += 1
    return H


def zstats_gpu_to_full(z):
    """GPU [44][n] statistics -> (g [n, 9], H [n, 9, 9], w [n]) in the oracle's z ordering."""
    n = z.shape[1]
    g = np.zeros((n, 9))
    H = np.zeros((n, 9, 9))
    g[:, 0:5] = z[0:5].T
    g[:, 5] = z[5]
    g[:, 6:9] = z[6:9].T
    H[:, :5, :5] = sym_from_packed(z[9:24], 5)
    for i in range(5):
        for ch in range(3):
            H[:, i, 6 + ch] = H[:, 6 + ch, i] = z[24 + i * 3 + ch]
    for ch in range(3):
        H[:, 6 + ch, 6 + ch] = z[39 + ch]
    H[:, 5, 5] = z[42]
    return g, H, z[43]


def blocks_gpu_to_oracle_view(blk, slot):
    """GPU blocks rows [35 + 10 V][n] -> oracle per-view layout [n, 56] for one single-view accumulation."""
    n = blk.shape[1]
    out = np.zeros((n, 56))
    out[:, 0:3] = blk[0:3].T
    out[:, 3:12] = sym_from_packed(blk[3:9], 3).reshape(n, 9)
    out[:, 12:16] = blk[9:13].T
    out[:, 16:32] = sym_from_packed(blk[13:23], 4).reshape(n, 16)
    out[:, 32:35] = blk[23:26].T
    out[:, 35:44] = sym_from_packed(blk[26:32], 3).reshape(n, 9)
    out[:, 44] = blk[32]
    out[:, 45] = blk[33]
    vb = 35 + 10 * slot
    out[:, 46] = blk[vb + 9]
    out[:, 47:50] = blk[vb:vb + 3].T
    out[:, 50:53] = blk[vb + 3:vb + 6].T
    out[:, 53:56] = blk[vb + 6:vb + 9].T
    return out


BLOCK_GROUPS = {
    "g_p": slice(0, 3), "H_p": slice(3, 12), "g_q": slice(12, 16), "H_q": slice(16, 32),
    "g_s": slice(32, 35), "H_s": slice(35, 44), "g_sigma": slice(44, 45), "H_sigma": slice(45, 46),
    "coverage": slice(46, 47), "gamma": slice(47, 50), "s_colour": slice(50, 53),
}
STEP_GROUPS = {"position": slice(0, 3), "rotation": slice(3, 4), "scale": slice(7, 10), "opacity": slice(10, 11)}


def gpu_view(ctx, gsn, dg, cam, target_t, lam, blocks, slot, keep=True):
    """Render + accumulate one view on the GPU; returns numpy copies of every stage."""
    import torch
    fr = ctx.frame()
    ccam = gsn.camera(cam)
    ro = gsn.render_opts()
    rgb = torch.zeros(3, cam.height, cam.width, dtype=torch.float32, device=ctx.device)
    T = torch.zeros(cam.height, cam.width, dtype=torch.float32, device=ctx.device)
    ctx.render(dg, ccam, ro, fr, rgb, T)
    loss = torch.zeros(2, dtype=torch.float64, device=ctx.device)
    ctx.accumulate_hessian(dg, fr, target_t, gsn.loss_opts(lam, 1.0, keep), slot, blocks, loss)
    torch.cuda.synchronize()
    ranges, ids, depth, rect, nc = fr.lists(dg.n, cam.width * cam.height)
    dL, h = fr.loss_maps(cam.height, cam.width)
    out = dict(img=rgb.cpu().numpy(), T=T.cpu().numpy(), ranges=ranges.cpu().numpy().astype(np.int64),
               ids=ids.cpu().numpy().view(np.uint32).astype(np.int64),
               depth=depth.cpu().numpy().view(np.uint32), rect=rect.cpu().numpy(),
               ncontrib=nc.cpu().numpy().reshape(cam.height, cam.width), dL=dL.cpu().numpy(), h=h.cpu().numpy(),
               loss=loss.cpu().numpy(), pairs=fr.info()[0])
    if keep:
        out["z"] = fr.zstats(dg.n).cpu().numpy()
    fr.close()
    return out


def oracle_view(g, cam, target, lam, o=None):
    o = O.opts(lambda_ssim=lam) if o is None else o
    fr = O.render(g, cam, o, g32=g)
    parts, dL, hd = O.loss(fr.img, target, lam)
    B = O.blocks(g, fr, dL, hd)
    Z = O.zstats(g, fr, dL, hd)
    return dict(fr=fr, parts=parts, dL=dL, hd=hd, blocks=B, z=Z)


def compare_binning(gv, ov, n):
    """Bit-exact comparison of depth keys, rectangles and per-tile lists; returns the number of tiles."""
    fr = ov["fr"]
    vis = fr.vis.astype(bool)
    assert np.array_equal(gv["depth"][vis], fr.depth[vis]), "depth keys differ"
    assert np.array_equal(gv["rect"][:, vis], fr.rect[:, vis]), "tile rectangles differ"
    assert np.all(gv["rect"][:, ~vis] == 0)
    ts = fr.tile_start
    assert gv["pairs"] == ts[-1], (gv["pairs"], ts[-1])
    ntiles = len(ts) - 1
    rg = gv["ranges"]
    for t in range(ntiles):
        a, b = rg[t]
        want = fr.ids[ts[t]:ts[t + 1]]
        got = gv["ids"][a:b] if b > a else np.zeros(0, np.int64)
        assert np.array_equal(got, want), f"tile {t}: list differs"
    return ntiles


def pixel_mask(ov, margin=MARGIN):
    return ov["fr"].margin >= margin
