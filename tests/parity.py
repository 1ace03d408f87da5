"""Shared helpers of the GPU parity tests: run one view through the HIP library
(C ABI via the ctypes binding) and through the FP64 oracle, and compare."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

# Tolerances (relative infinity norm per tensor / per attribute group).
TOL_IMAGE = 1e-5
TOL_GRAD = 1e-5
TOL_STEP = 1e-4
# Oracle pixels whose threshold decisions (alpha_min, alpha_max, T_min) sit within this relative
# distance of the threshold are not compared element-wise: ten times the single-precision error of
# alpha and of the transmittance product, so the two sides may take such a decision differently.
MARGIN = 1e-5


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
    """GPU blocks rows [30 + 10 V + 1][n] -> oracle per-view layout [n, 49] for one single-view accumulation."""
    n = blk.shape[1]
    V = (blk.shape[0] - 31) // 10
    out = np.zeros((n, 49))
    out[:, 0:3] = blk[0:3].T
    out[:, 3:12] = sym_from_packed(blk[3:9], 3).reshape(n, 9)
    out[:, 12:15] = blk[9:12].T
    out[:, 15:24] = sym_from_packed(blk[12:18], 3).reshape(n, 9)
    out[:, 24:27] = blk[18:21].T
    out[:, 27:36] = sym_from_packed(blk[21:27], 3).reshape(n, 9)
    out[:, 36] = blk[27]
    out[:, 37] = blk[28]
    vb = 30 + 10 * slot
    out[:, 38] = blk[vb + 9]
    out[:, 39:42] = blk[vb:vb + 3].T
    out[:, 42:45] = blk[vb + 3:vb + 6].T
    out[:, 45:48] = blk[vb + 6:vb + 9].T
    out[:, 48] = blk[30 + 10 * V]
    return out


BLOCK_GROUPS = {
    "g_p": slice(0, 3), "H_p": slice(3, 12), "g_omega": slice(12, 15), "H_omega": slice(15, 24),
    "g_s": slice(24, 27), "H_s": slice(27, 36), "g_sigma": slice(36, 37), "H_sigma": slice(37, 38),
    "coverage": slice(38, 39), "gamma": slice(39, 42), "s_colour": slice(42, 45), "w2": slice(48, 49),
}
STEP_GROUPS = {"position": slice(0, 3), "rotation": slice(3, 4), "scale": slice(7, 10), "opacity": slice(10, 11)}


def gpu_view(ctx, gsn, dg, cam, target_t, lam, blocks, slot, keep=True, gn=False, precision=0, render_precision=0):
    """Render + accumulate one view on the GPU; returns numpy copies of every stage."""
    import torch
    fr = ctx.frame()
    ccam = cam if isinstance(cam, gsn.CCamera) else gsn.camera(cam)
    ro = gsn.render_opts(precision=render_precision)
    rgb = torch.zeros(3, cam.height, cam.width, dtype=torch.float32, device=ctx.device)
    T = torch.zeros(cam.height, cam.width, dtype=torch.float32, device=ctx.device)
    ctx.render(dg, ccam, ro, fr, rgb, T)
    loss = torch.zeros(2, dtype=torch.float64, device=ctx.device)
    ctx.accumulate_hessian(dg, fr, target_t, gsn.loss_opts(lam, 1.0, keep, gn, precision), slot, blocks, loss)
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
        out["rec"] = fr.records(dg.n).cpu().numpy()
    fr.close()
    return out


def oracle_view(g, cam, target, lam, o=None, gn=False):
    o = O.opts(lambda_ssim=lam, gauss_newton=int(gn)) if o is None else o
    fr = O.render(g, cam, o, g32=g)
    parts, dL, hd = O.loss(fr.img, target, lam)
    B = O.blocks(g, fr, dL, hd)
    Z = O.zstats(g, fr, dL, hd)
    return dict(fr=fr, parts=parts, dL=dL, hd=hd, blocks=B, z=Z)


def view_errors(g, cam, gv, ov, blk):
    """Per-stage relative errors of one GPU view (gpu_view, its single-view blocks) against the oracle's
    (oracle_view), on the pixels and kernels whose decisions are unambiguous; returns (errors, kept kernels)."""
    mask = pixel_mask(ov)
    errs = {"ambiguous_px": int((~mask).sum())}
    fr = ov["fr"]
    errs["img"] = rel_inf(gv["img"][:, mask], fr.img[:, mask])
    errs["T"] = rel_inf(gv["T"][mask], fr.Tfinal[mask])
    errs["ncontrib_mismatch"] = int((gv["ncontrib"][mask] != fr.ncontrib[mask]).sum())
    errs["loss_L2"] = abs(gv["loss"][0] - ov["parts"][0]) / abs(ov["parts"][0])
    errs["loss_S"] = abs(gv["loss"][1] - ov["parts"][1]) / abs(ov["parts"][1])
    # loss maps beyond the SSIM reach of the ambiguous pixels (their windows carry an ambiguous
    # pixel's legitimate difference into the neighbours' derivatives)
    reach = ssim_reach(mask)
    errs["dL"] = rel_inf(gv["dL"][:, ~reach], ov["dL"][:, ~reach])
    errs["h"] = rel_inf(gv["h"][:, ~reach], ov["hd"][:, ~reach])
    # kernels composited at an ambiguous pixel or within its reach are excluded from the
    # per-kernel comparisons
    bad = near_threshold_kernels(fr, g.n) | kernels_in_reach(fr, reach, g.n)
    errs["excluded_kernels"] = int(bad.sum())
    keep = ~bad
    gz, Hz, wz = zstats_gpu_to_full(gv["z"])
    # the oracle's statistics in each kernel's principal frame, taken from the oracle's own projection
    fc, fs = oracle_frames(g, cam)
    Zo = zstats_to_frame(ov["z"], fc, fs)
    errs["z_g"] = rel_inf(gz[keep], Zo[keep, :9])
    # the library keeps the (pi, Q, c~) block and the sigma-sigma entry: the sigma cross terms
    # are not needed by any attribute group (no attribute moves both sigma and pi, Q or c~)
    used = np.zeros((9, 9), bool)
    used[:5, :5] = used[:5, 6:] = used[6:, :5] = True
    used[5, 5] = True
    used[[6, 7, 8], [6, 7, 8]] = True
    errs["z_H"] = rel_inf(Hz[keep][:, used], Zo[keep, 9:90].reshape(-1, 9, 9)[:, used])
    errs["z_w"] = rel_inf(wz[keep], Zo[keep, 90])
    Bg = blocks_gpu_to_oracle_view(blk, 0)
    for name, sl in BLOCK_GROUPS.items():
        errs[name] = rel_inf(Bg[keep][:, sl], ov["blocks"][keep][:, sl])
    return errs, keep


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


def near_threshold_kernels(fr, n, margin=MARGIN):
    """Kernels composited (up to and including the stopping entry) at any pixel whose oracle
    threshold decisions sit within `margin` of a threshold; their statistics may legitimately
    differ between single- and double-precision compositing."""
    bad = np.zeros(n, bool)
    amb = fr.margin < margin
    if fr.tile_start is None or not amb.any():
        return bad
    tx = (fr.cam.width + 15) // 16
    for y, x in zip(*np.nonzero(amb)):
        t = (y // 16) * tx + x // 16
        lst = fr.ids[fr.tile_start[t]:fr.tile_start[t + 1]]
        bad[lst[:int(fr.ncontrib[y, x]) + 1]] = True
    return bad


def ssim_reach(mask, radius=10):
    """Pixels within `radius` (the SSIM window's reach: a window of radius 5 around each window
    centre of radius 5) of a pixel outside `mask`; their loss derivatives depend on it."""
    from scipy.ndimage import binary_dilation
    return binary_dilation(~mask, structure=np.ones((2 * radius + 1, 2 * radius + 1), bool))


def kernels_in_reach(fr, reach, n):
    """Kernels that may composite at a pixel of `reach`: per tile, the list prefix up to the
    longest such pixel's last composited entry."""
    bad = np.zeros(n, bool)
    if fr.tile_start is None or not reach.any():
        return bad
    tx = (fr.cam.width + 15) // 16
    ys, xs = np.nonzero(reach)
    deepest = np.full(len(fr.tile_start) - 1, -1, np.int64)
    np.maximum.at(deepest, (ys // 16) * tx + xs // 16, fr.ncontrib[ys, xs].astype(np.int64))
    for t in np.nonzero(deepest >= 0)[0]:
        bad[fr.ids[fr.tile_start[t]:fr.tile_start[t] + deepest[t] + 1]] = True
    return bad


def zstats_to_frame(Z, fc, fs):
    """Oracle statistics [n, 91] over (pi_x, pi_y, Q_xx, Q_xy, Q_yy, sigma, c~) -> the same in each
    kernel's principal frame (pi' = V^T pi, Q' = V^T Q V, V = [[c, -s], [s, c]])."""
    n = Z.shape[0]
    g = Z[:, :9].copy()
    H = Z[:, 9:90].reshape(n, 9, 9).copy()
    L = np.zeros((n, 9, 9))
    c, s = np.asarray(fc, np.float64), np.asarray(fs, np.float64)
    L[:, 0, 0], L[:, 0, 1], L[:, 1, 0], L[:, 1, 1] = c, -s, s, c
    # (Q_xx, Q_xy, Q_yy) = Lq (Q'_11, Q'_12, Q'_22) for Q = V Q' V^T
    L[:, 2, 2], L[:, 2, 3], L[:, 2, 4] = c * c, -2 * c * s, s * s
    L[:, 3, 2], L[:, 3, 3], L[:, 3, 4] = c * s, c * c - s * s, -c * s
    L[:, 4, 2], L[:, 4, 3], L[:, 4, 4] = s * s, 2 * c * s, c * c
    for i in range(5, 9):
        L[:, i, i] = 1.0
    gl = np.einsum("nij,ni->nj", L, g)
    Hl = np.einsum("nia,nij,njb->nab", L, H, L)
    out = Z.copy()
    out[:, :9] = gl
    out[:, 9:90] = Hl.reshape(n, 81)
    return out


def gpu_blocks_to_summed(gb, V):
    """GPU blocks rows [30 + 10 V + 1][n] -> the oracle's summed solve layout [n][39 + 10 V + 1]."""
    n = gb.shape[1]
    S = np.zeros((n, 40 + 10 * V))
    S[:, 0:3] = gb[0:3].T
    S[:, 3:12] = sym_from_packed(gb[3:9], 3).reshape(n, 9)
    S[:, 12:15] = gb[9:12].T
    S[:, 15:24] = sym_from_packed(gb[12:18], 3).reshape(n, 9)
    S[:, 24:27] = gb[18:21].T
    S[:, 27:36] = sym_from_packed(gb[21:27], 3).reshape(n, 9)
    S[:, 36], S[:, 37], S[:, 38] = gb[27], gb[28], gb[29]
    for v in range(V):
        S[:, 39 + 10 * v:49 + 10 * v] = gb[30 + 10 * v:40 + 10 * v].T
    S[:, 39 + 10 * V] = gb[30 + 10 * V]
    return S


def packed_from_sym(M):
    """[n, 3, 3] symmetric -> packed upper triangle rows [6][n] (row by row)."""
    return np.stack([M[:, i, j] for i in range(3) for j in range(i, 3)])


def summed_to_gpu_blocks(S, V):
    """The oracle's summed solve layout [n][39 + 10 V + 1] -> the library's block rows [30 + 10 V + 1][n]."""
    n = S.shape[0]
    gb = np.zeros((31 + 10 * V, n))
    gb[0:3] = S[:, 0:3].T
    gb[3:9] = packed_from_sym(S[:, 3:12].reshape(n, 3, 3))
    gb[9:12] = S[:, 12:15].T
    gb[12:18] = packed_from_sym(S[:, 15:24].reshape(n, 3, 3))
    gb[18:21] = S[:, 24:27].T
    gb[21:27] = packed_from_sym(S[:, 27:36].reshape(n, 3, 3))
    gb[27], gb[28], gb[29] = S[:, 36], S[:, 37], S[:, 38]
    for v in range(V):
        gb[30 + 10 * v:40 + 10 * v] = S[:, 39 + 10 * v:49 + 10 * v].T
    gb[30 + 10 * V] = S[:, 39 + 10 * V]
    return gb


def oracle_frames(g, cam, kappa=0.3):
    """Principal frame (c, s) of each kernel's FP64 projected covariance: e1 = (c, s) is the
    eigenvector of the larger eigenvalue, picked from the better conditioned of the two
    eigenvector formulas (the convention the library's records state)."""
    out, _ = O.project64(g, cam, kappa=kappa)
    sxx, sxy, syy = out[:, 2], out[:, 3], out[:, 4]
    half = 0.5 * (sxx - syy)
    l1 = 0.5 * (sxx + syy) + np.sqrt(half * half + sxy * sxy)
    vx, vy = l1 - syy, sxy.copy()
    alt = np.abs(sxy) + np.abs(l1 - sxx) > np.abs(vx) + np.abs(vy)
    vx = np.where(alt, sxy, vx)
    vy = np.where(alt, l1 - sxx, vy)
    nn = np.hypot(vx, vy)
    safe = np.where(nn > 0, nn, 1.0)
    return np.where(nn > 0, vx / safe, 1.0), np.where(nn > 0, vy / safe, 0.0)


def _block_groups(V):
    """Column groups of the oracle's summed layout whose entries are sums of the same per-pixel
    terms: a float32 sum is accurate to a fraction of the group's largest entry, not of each entry
    (a small entry can be the cancelled remainder of large terms)."""
    groups = [slice(0, 3), slice(3, 12), slice(12, 15), slice(15, 24), slice(24, 27), slice(27, 36),
              slice(36, 37), slice(37, 38), slice(38, 39)]
    for v in range(V):
        b = O.NB_BASE + O.NB_VIEW * v
        groups += [slice(b, b + 3), slice(b + 3, b + 6), slice(b + 6, b + 9), slice(b + 9, b + 10)]
    return groups


def step_sensitivity(g, cam, o, summed, V, rel=1e-5, trials=4, seed=0):
    """Per kernel and group, the largest change of the oracle's step when its inputs carry
    noise `rel` times the largest entry of each kernel's block (the precision the blocks are
    required to have), divided by the group's largest step: how precisely the step is
    determined by blocks of that accuracy."""
    rng = np.random.default_rng(seed)
    base, dec = O.solve(g, cam, o, summed, V)
    dev = np.zeros((summed.shape[0], len(STEP_GROUPS) + 1))
    scale = np.zeros_like(summed)
    for sl in _block_groups(V):
        scale[:, sl] = np.max(np.abs(summed[:, sl]), axis=1, keepdims=True)
    for _ in range(trials):
        noisy = summed + rel * scale * rng.standard_normal(summed.shape)
        st, _ = O.solve(g, cam, o, noisy, V)
        for i, sl in enumerate(list(STEP_GROUPS.values()) + [slice(11, None)]):
            den = max(np.max(np.abs(base[:, sl])), 1e-300)
            dev[:, i] = np.maximum(dev[:, i], np.max(np.abs(st[:, sl] - base[:, sl]), axis=1) / den)
    return dev
