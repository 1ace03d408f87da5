"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It loads ``liboracle.so`` built from
``gsn_oracle.cpp`` (see :func:`build`) and composes its routines into the
per-image local-Newton sweep of the paper (Sec. 4.2-4.3):

  primary target: project -> bin -> composite -> loss maps -> per-kernel blocks
  each secondary target (KNN camera at half resolution): the same, blocks added
  reduced-coordinate damped solves -> apply (position, rotation, scaling,
  opacity, colour).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gsn_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

O_NAMES = ["tile", "alpha_min", "alpha_max", "T_min", "kappa", "radius_sigma", "smooth",
           "bg_r", "bg_g", "bg_b", "lambda_ssim", "barrier_beta", "damp_rel", "damp_abs",
           "pivot_min", "max_esc", "sh_floor", "scale_floor", "opac_ftb", "npix_primary", "trust_pos",
           "trust_rot", "trust_scale", "trust_sh", "opac_eps", "step_frac", "damp_sh", "gauss_newton",
           "overlap"]
DEFAULTS = dict(tile=16, alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, kappa=0.3,
                radius_sigma=3.0, smooth=0, bg_r=0.0, bg_g=0.0, bg_b=0.0, lambda_ssim=0.2,
                barrier_beta=1e-2, damp_rel=1e-3, damp_abs=1e-12, pivot_min=1e-3, max_esc=7,
                sh_floor=1e-3, scale_floor=0.1, opac_ftb=0.995, npix_primary=1.0, trust_pos=2.0,
                trust_rot=0.5, trust_scale=0.5, trust_sh=1.0, opac_eps=1e-6, step_frac=1.0,
                damp_sh=1e-3, gauss_newton=0, overlap=0)
B_COUNT = 49
NB_BASE, NB_VIEW = 39, 10


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP contraction off so the FP32 spec is exact)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "jet.hpp"))):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def opts(**kw) -> np.ndarray:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return np.array([float(d[k]) for k in O_NAMES], np.float64)


def cam_vec(cam, dtype=np.float64) -> np.ndarray:
    v = np.zeros(20, dtype)
    v[0:9] = np.asarray(cam.R, np.float32).reshape(-1)
    v[9:12] = np.asarray(cam.t, np.float32)
    v[12:19] = [cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.znear]
    if dtype == np.float32:
        v = v.astype(np.float32)
    else:
        # the FP64 stages see exactly the float32 camera values
        v[12:16] = np.asarray(v[12:16], np.float32)
        v[18] = np.float32(v[18])
    return v


@dataclass
class G64:
    """Kernel parameters in float64 (converted exactly from the float32 inputs)."""
    pos: np.ndarray
    rot: np.ndarray
    scale: np.ndarray
    opac: np.ndarray
    sh: np.ndarray
    K: int

    @property
    def n(self):
        return self.pos.shape[1]

    @staticmethod
    def of(g):
        if isinstance(g, G64):
            return g
        c = lambda a: np.ascontiguousarray(a, np.float64)  # noqa: E731
        return G64(c(g.pos), c(g.rot), c(g.scale), c(g.opac), c(g.sh), int(g.sh.shape[1]))

    def copy(self):
        return G64(self.pos.copy(), self.rot.copy(), self.scale.copy(), self.opac.copy(),
                   self.sh.copy(), self.K)

    def args(self):
        return (ctypes.c_int(self.n), ctypes.c_int(self.K), _p(self.pos), _p(self.rot),
                _p(self.scale), _p(self.opac), _p(self.sh))


def sh_basis(K: int, r) -> np.ndarray:
    out = np.zeros(K, np.float64)
    lib().orc_sh_basis(ctypes.c_int(K), _p(np.ascontiguousarray(r, np.float64)), _p(out))
    return out


def tiles_of(cam, tile=16):
    return (cam.width + tile - 1) // tile, (cam.height + tile - 1) // tile


def project32(g, cam, o):
    """FP32 binning decisions: depth bits [N] u32, rect [4][N] i32 (x0,y0,x1,y1), visible [N] u8."""
    n = g.pos.shape[1]
    f = lambda a: np.ascontiguousarray(a, np.float32)  # noqa: E731
    pos, rot, scale = f(g.pos), f(g.rot), f(g.scale)
    depth = np.zeros(n, np.uint32)
    rect = np.zeros((4, n), np.int32)
    vis = np.zeros(n, np.uint8)
    kappa = 0.0 if o[O_NAMES.index("smooth")] else o[O_NAMES.index("kappa")]
    lib().orc_project32(ctypes.c_int(n), _p(pos), _p(rot), _p(scale), _p(cam_vec(cam, np.float32)),
                        ctypes.c_float(kappa), ctypes.c_float(o[O_NAMES.index("radius_sigma")]),
                        ctypes.c_int(int(o[0])), _p(depth), _p(rect), _p(vis))
    return depth, rect, vis


def tile_lists(depth, rect, vis, tiles_x, tiles_y):
    n = depth.shape[0]
    ts = np.zeros(tiles_x * tiles_y + 1, np.int64)
    L = lib()
    L.orc_tile_lists.restype = ctypes.c_int64
    total = L.orc_tile_lists(ctypes.c_int(n), _p(depth), _p(rect), _p(vis), ctypes.c_int(tiles_x),
                             ctypes.c_int(tiles_y), _p(ts), None)
    ids = np.zeros(max(total, 1), np.int32)
    L.orc_tile_lists(ctypes.c_int(n), _p(depth), _p(rect), _p(vis), ctypes.c_int(tiles_x),
                     ctypes.c_int(tiles_y), _p(ts), _p(ids))
    return ts, ids[:total]


@dataclass
class Frame:
    cam: object
    o: np.ndarray
    depth: np.ndarray = None
    rect: np.ndarray = None
    vis: np.ndarray = None
    tile_start: np.ndarray = None
    ids: np.ndarray = None
    img: np.ndarray = None
    Tfinal: np.ndarray = None
    ncontrib: np.ndarray = None
    margin: np.ndarray = None


def render(g, cam, o, g32=None) -> Frame:
    """FP64 render.  Standard mode bins with the FP32 spec of ``g32`` (default: g rounded to f32)."""
    g64 = G64.of(g)
    fr = Frame(cam, o)
    smooth = bool(o[O_NAMES.index("smooth")])
    if not smooth:
        src = g32 if g32 is not None else g64
        fr.depth, fr.rect, fr.vis = project32(src, cam, o)
        tx, ty = tiles_of(cam, int(o[0]))
        fr.tile_start, fr.ids = tile_lists(fr.depth, fr.rect, fr.vis, tx, ty)
    H, W = cam.height, cam.width
    fr.img = np.zeros((3, H, W))
    fr.Tfinal = np.zeros((H, W))
    fr.ncontrib = np.zeros((H, W), np.int32)
    fr.margin = np.zeros((H, W))
    lib().orc_render(*g64.args(), _p(cam_vec(cam)), _p(o), _p(fr.tile_start), _p(fr.ids),
                     _p(fr.img), _p(fr.Tfinal), _p(fr.ncontrib), _p(fr.margin))
    return fr


def loss(img, tgt, lam, derivs=True):
    """Returns (L2, L_S), dL [3][H][W], hdiag [3][H][W]; L = L2 + lam * L_S."""
    img = np.ascontiguousarray(img, np.float64)
    tgt = np.ascontiguousarray(tgt, np.float64)
    _, H, W = img.shape
    parts = np.zeros(2)
    dL = np.zeros_like(img) if derivs else None
    hd = np.zeros_like(img) if derivs else None
    lib().orc_loss(ctypes.c_int(W), ctypes.c_int(H), _p(img), _p(tgt), ctypes.c_double(lam),
                   _p(dL), _p(hd), _p(parts))
    return (parts[0], parts[1]), dL, hd


def blocks(g, fr: Frame, dL, hd, sel=None):
    g64 = G64.of(g)
    sel = np.arange(g64.n, dtype=np.int32) if sel is None else np.ascontiguousarray(sel, np.int32)
    out = np.zeros((len(sel), B_COUNT))
    rect = fr.rect if fr.rect is not None else np.zeros((4, g64.n), np.int32)
    lib().orc_blocks(*g64.args(), _p(cam_vec(fr.cam)), _p(fr.o), _p(fr.tile_start), _p(fr.ids),
                     _p(rect), _p(np.ascontiguousarray(dL)), _p(np.ascontiguousarray(hd)),
                     ctypes.c_int(len(sel)), _p(sel), _p(out))
    return out


def zstats(g, fr: Frame, dL, hd, sel=None):
    g64 = G64.of(g)
    sel = np.arange(g64.n, dtype=np.int32) if sel is None else np.ascontiguousarray(sel, np.int32)
    out = np.zeros((len(sel), 91))
    rect = fr.rect if fr.rect is not None else np.zeros((4, g64.n), np.int32)
    lib().orc_zstats(*g64.args(), _p(cam_vec(fr.cam)), _p(fr.o), _p(fr.tile_start), _p(fr.ids),
                     _p(rect), _p(np.ascontiguousarray(dL)), _p(np.ascontiguousarray(hd)),
                     ctypes.c_int(len(sel)), _p(sel), _p(out))
    return out


def sum_blocks(per_view):
    """Combine per-view blocks [V] of [n][49] into the solve layout [n][39 + 10 V + 1].

    Position, rotation, scaling and opacity blocks are summed over the views
    (weight 1, Sec. 4.3); the colour statistics stay per view; the coverage
    of the first (primary) view decides which kernels are trained; the last
    column sums sum_pix (alpha T)^2 over the views (the overlap share's numerator)."""
    V = len(per_view)
    n = per_view[0].shape[0]
    out = np.zeros((n, NB_BASE + NB_VIEW * V + 1))
    for b in per_view:
        out[:, :38] += b[:, :38]
    out[:, 38] = per_view[0][:, 38]
    for v, b in enumerate(per_view):
        base = NB_BASE + NB_VIEW * v
        out[:, base:base + 3] = b[:, 39:42]
        out[:, base + 3:base + 6] = b[:, 42:45]
        out[:, base + 6:base + 9] = b[:, 45:48]
        out[:, base + 9] = b[:, 38]
    out[:, NB_BASE + NB_VIEW * V] = sum(b[:, 48] for b in per_view)
    return out


def solve(g, cam, o, summed, V, with_cond=False):
    """Reduced-coordinate damped solves; returns steps [n][11 + 3K], decisions [n][5] (and
    the condition number [n][4] of each group's solved matrix when with_cond)."""
    g64 = G64.of(g)
    K = g64.K
    steps = np.zeros((g64.n, 11 + 3 * K))
    dec = np.zeros((g64.n, 5), np.int32)
    cond = np.zeros((g64.n, 4))
    lib().orc_solve(ctypes.c_int(g64.n), ctypes.c_int(K), _p(g64.pos), _p(g64.rot), _p(g64.scale),
                    _p(g64.opac), _p(cam_vec(cam)), _p(o), ctypes.c_int(V),
                    _p(np.ascontiguousarray(summed)), _p(steps), _p(dec), _p(cond))
    return (steps, dec, cond) if with_cond else (steps, dec)


def apply(g, steps, dec, o, mask=31, scale=None) -> G64:
    """Applies the steps; scale [n][5] (optional) multiplies each group's step of each kernel
    (position, rotation angle, scaling, opacity, colour) before it is applied."""
    out = G64.of(g).copy()
    if scale is not None:
        steps = np.array(steps, np.float64)
        sc = np.asarray(scale, np.float64)
        K = out.K
        for gi, sl in enumerate([slice(0, 3), slice(3, 4), slice(7, 10), slice(10, 11), slice(11, 11 + 3 * K)]):
            steps[:, sl] *= sc[:, gi:gi + 1]
    lib().orc_apply(ctypes.c_int(out.n), ctypes.c_int(out.K), _p(out.pos), _p(out.rot), _p(out.scale),
                    _p(out.opac), _p(out.sh), _p(o), _p(np.ascontiguousarray(steps)),
                    _p(np.ascontiguousarray(dec)), ctypes.c_int(mask))
    return out


def knn(centers, scene_center, K=3):
    centers = np.ascontiguousarray(centers, np.float64)
    out = np.zeros((centers.shape[0], K), np.int32)
    lib().orc_knn(ctypes.c_int(centers.shape[0]), _p(centers),
                  _p(np.ascontiguousarray(scene_center, np.float64)), ctypes.c_int(K), _p(out))
    return out


def camera_knn(cams, g, K=3):
    centers = np.stack([c.center for c in cams])
    scene_center = np.asarray(g.pos, np.float64).mean(axis=1)
    return knn(centers, scene_center, K)


def half_camera(cam):
    """Camera of a secondary target (Sec. 4.3, reading C17): the image is the 2x2 box
    mean of the full-resolution one, so a half-resolution pixel centre (integer
    coordinate u') sits at the full-resolution coordinate 2 u' + 0.5; focal lengths are
    halved and the principal point maps as c' = (c + 0.5) / 2 - 0.5.  Values are
    rounded to float32 like every camera input."""
    from synth.scenes import Camera
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    return Camera(np.array(cam.R, np.float32), np.array(cam.t, np.float32),
                  f32(0.5 * float(cam.fx)), f32(0.5 * float(cam.fy)),
                  f32(0.5 * (float(cam.cx) + 0.5) - 0.5), f32(0.5 * (float(cam.cy) + 0.5) - 0.5),
                  cam.width // 2, cam.height // 2, cam.znear)


def downsample(img):
    img = np.ascontiguousarray(img, np.float64)
    _, H, W = img.shape
    out = np.zeros((3, H // 2, W // 2))
    lib().orc_downsample(ctypes.c_int(W), ctypes.c_int(H), _p(img), _p(out))
    return out


def view_blocks(g, cam, target, o, sel=None):
    """Render one view, its loss maps and the per-kernel blocks.  Returns (frame, loss parts, blocks)."""
    fr = render(g, cam, o)
    parts, dL, hd = loss(fr.img, target, o[O_NAMES.index("lambda_ssim")])
    return fr, parts, blocks(g, fr, dL, hd, sel)


def sweep(g, cams, targets, t, knn_table=None, o=None, mask=31):
    """One stochastic local-Newton sweep for training image t (Sec. 4.2-4.3).

    The primary target is view t at full resolution; each KNN secondary is
    rendered at half resolution against its 2x2 box-downsampled target.
    All groups are linearised at the same state and applied in the order
    position, rotation, scaling, opacity, colour.  Returns a dict."""
    g64 = G64.of(g)
    cam = cams[t]
    o = opts() if o is None else o.copy()
    o[O_NAMES.index("npix_primary")] = cam.width * cam.height
    views = [(cam, np.asarray(targets[t], np.float64))]
    if knn_table is not None:
        for j in knn_table[t]:
            views.append((half_camera(cams[j]), downsample(targets[j])))
    per_view, losses, frames = [], [], []
    for c, tg in views:
        fr, parts, b = view_blocks(g64, c, tg, o)
        per_view.append(b)
        losses.append(parts)
        frames.append(fr)
    summed = sum_blocks(per_view)
    steps, dec, cond = solve(g64, cam, o, summed, len(views), with_cond=True)
    new = apply(g64, steps, dec, o, mask)
    return dict(new=new, steps=steps, dec=dec, cond=cond, summed=summed, per_view=per_view,
                losses=losses, frames=frames, opts=o)


def sweep_series(g, cams, targets, t, knn_table=None, o=None, order=(1, 2, 4, 8, 16)):
    """Series schedule (Sec. 4.2): one sweep per group mask in `order`, each linearised at the
    state the previous groups left and applying only its own group.  Returns the final state
    and the per-stage sweep results."""
    stages = []
    for m in order:
        res = sweep(g, cams, targets, t, knn_table, o, m)
        stages.append(res)
        g = res["new"]
    return g, stages


def psnr(img, tgt):
    a = np.clip(np.asarray(img, np.float64), 0.0, 1.0)
    mse = float(np.mean((a - np.asarray(tgt, np.float64)) ** 2))
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else float("inf")


def project64(g, cam, kappa=0.3):
    """FP64 projection per kernel: [n][12] (pi 2, Sigma 3, Q 3, c~ 3, depth) and ok [n]."""
    g64 = G64.of(g)
    out = np.zeros((g64.n, 12))
    ok = np.zeros(g64.n, np.uint8)
    lib().orc_project64(*g64.args(), _p(cam_vec(cam)), ctypes.c_double(kappa), _p(out), _p(ok))
    return out, ok


def render_z(recs, W, H, bg=(0.0, 0.0, 0.0)):
    """Smooth composite of projected records [n][10] (pi, Q, sigma, c~, depth)."""
    recs = np.ascontiguousarray(recs, np.float64)
    img = np.zeros((3, H, W))
    lib().orc_render_z(ctypes.c_int(recs.shape[0]), _p(recs), ctypes.c_int(W), ctypes.c_int(H),
                       _p(np.asarray(bg, np.float64)), _p(img))
    return img
