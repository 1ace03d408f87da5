"""ctypes binding of libgsn (include/gsn.h): argument marshalling only.

Every step of the training path runs in the HIP library; this module turns
torch device tensors into the plain pointers and structs of the C ABI.  It
raises if the library has not been built -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsn.so")

GSN_BLK_BASE, GSN_BLK_VIEW, GSN_STEP_BASE, GSN_NZ = 30, 10, 11, 48
GSN_FEAT_HIDDEN, GSN_FEAT_OK, GSN_FEAT_OUT_OF_RANGE = 0, 1, 2
STATUS = {0: "GSN_OK", -1: "GSN_E_INVALID", -2: "GSN_E_SHAPE", -3: "GSN_E_CAPACITY", -4: "GSN_E_HIP",
          -5: "GSN_E_NOMEM", -6: "GSN_E_NUMERIC"}
GSN_E_CAPACITY, GSN_E_NUMERIC = -3, -6
STATS = ("culled_nonfinite", "skipped_nonfinite", "pair_overflow", "pairs_needed")

_lib = None


class GsnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python paper_2501_13975_amd/build_lib.py)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        for name, args in {
            "gsn_create": [ctypes.POINTER(P), ctypes.c_int32, P],
            "gsn_destroy": [P], "gsn_set_stream": [P, P],
            "gsn_frame_create": [P, ctypes.POINTER(P)], "gsn_frame_destroy": [P, P],
            "gsn_render": [P, P, P, P, P, P, P],
            "gsn_accumulate_hessian": [P, P, P, P, P, ctypes.c_int32, P, P],
            "gsn_accumulate_views": [P, P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_int32],
            "gsn_add_view_shares": [P, P, ctypes.c_int32, P],
            "gsn_local_newton_solve": [P, P, P, P, P, P],
            "gsn_local_newton_solve_noalloc": [P, P, P, P, P, P],
            "gsn_apply_step": [P, P, P, P, P, ctypes.c_uint32],
            "gsn_solve_apply": [P, P, P, P, P, P, ctypes.c_uint32],
            "gsn_first_order_step": [P, P, P, P, P, P, ctypes.c_uint32],
            "gsn_step_features": [P, P, P, P, P, P, P, P],
            "gsn_neighbour_residual": [P, P, P],
            "gsn_solve_batched": [P, P, ctypes.c_int32],
            "gsn_sh_gram": [P, P, ctypes.c_int32, P],
            "gsn_solve_tune": [P, P, ctypes.c_int32, P, P],
            "gsn_solve_graph_create": [P, P, ctypes.c_int32, ctypes.POINTER(P)],
            "gsn_graph_launch": [P, P], "gsn_graph_destroy": [P, P],
            "gsn_step_labels": [P, P, P, P, P, P, P, P],
            "gsn_mlp_reset": [P, P],
            "gsn_mlp_infer": [P, P, ctypes.c_int32, P, P, P, P],
            "gsn_mlp_train_step": [P, P, ctypes.c_int32, P, P, P, P, P, P],
            "gsn_blocks_zero": [P, P],
            "gsn_downsample2x": [P, P, ctypes.c_int32, ctypes.c_int32, P],
            "gsn_camera_knn": [P, ctypes.c_int32, P, ctypes.c_int32, P],
            "gsn_camera_half": [P, P],
            "gsn_scene_center": [P, P, P],
            "gsn_frame_info": [P, P, P, P, P],
            "gsn_frame_lists": [P, P, P, P, P, P, P],
            "gsn_frame_zstats": [P, P, P],
            "gsn_frame_loss_maps": [P, P, P, P],
            "gsn_frame_records": [P, P, P],
            "gsn_profile_enable": [P, ctypes.c_int32],
            "gsn_profile_read": [P, P, P, P],
            "gsn_sync_status": [P, P],
            "gsn_frame_reserve": [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64],
            "gsn_capture_begin": [P],
            "gsn_capture_end": [P, ctypes.POINTER(P)],
        }.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.gsn_last_error.argtypes = [P]
        L.gsn_last_error.restype = ctypes.c_char_p
        L.gsn_blocks_floats.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.gsn_blocks_floats.restype = ctypes.c_int64
        L.gsn_steps_floats.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.gsn_steps_floats.restype = ctypes.c_int64
        _lib = L
    return _lib


# ------------------------------------------------------------------ C structs
class CGaussians(ctypes.Structure):
    _fields_ = [("d_pos", ctypes.c_void_p), ("d_rot", ctypes.c_void_p), ("d_scale", ctypes.c_void_p),
                ("d_opac", ctypes.c_void_p), ("d_sh", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32)]


class CCamera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("znear", ctypes.c_float)]


class CRenderOpts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("T_min", ctypes.c_float), ("kappa", ctypes.c_float), ("radius_sigma", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("precision", ctypes.c_int32)]


class CLossOpts(ctypes.Structure):
    _fields_ = [("lambda_ssim", ctypes.c_float), ("weight", ctypes.c_float), ("keep_zstats", ctypes.c_int32),
                ("gauss_newton", ctypes.c_int32), ("precision", ctypes.c_int32)]


class CSolveOpts(ctypes.Structure):
    _fields_ = [("damp_rel", ctypes.c_float), ("damp_abs", ctypes.c_float), ("pivot_min", ctypes.c_float),
                ("max_escalations", ctypes.c_int32), ("barrier_beta", ctypes.c_float),
                ("sh_floor", ctypes.c_float), ("scale_floor", ctypes.c_float), ("opac_ftb", ctypes.c_float),
                ("npix_primary", ctypes.c_int32), ("kappa", ctypes.c_float), ("trust_pos", ctypes.c_float),
                ("trust_rot", ctypes.c_float), ("trust_scale", ctypes.c_float), ("trust_sh", ctypes.c_float),
                ("opac_eps", ctypes.c_float), ("step_frac", ctypes.c_float), ("damp_sh", ctypes.c_float),
                ("precision", ctypes.c_int32), ("overlap_scale", ctypes.c_int32), ("view_limit", ctypes.c_int32)]


class CBlocks(ctypes.Structure):
    _fields_ = [("d_data", ctypes.c_void_p), ("n", ctypes.c_int32), ("n_views", ctypes.c_int32)]


class CSteps(ctypes.Structure):
    _fields_ = [("d_data", ctypes.c_void_p), ("d_flags", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32)]


def render_opts(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, kappa=0.3, radius_sigma=3.0,
                bg=(0.0, 0.0, 0.0), precision=0):
    """precision 1: the mixed form's single-precision colour sums."""
    return CRenderOpts(16, alpha_min, alpha_max, T_min, kappa, radius_sigma, (ctypes.c_float * 3)(*bg),
                       int(precision))


def loss_opts(lambda_ssim=0.2, weight=1.0, keep_zstats=False, gauss_newton=False, precision=0):
    """precision 1: the mixed form's single-precision SSIM maps, statistic sums and rotation/scale chain."""
    return CLossOpts(lambda_ssim, weight, int(keep_zstats), int(gauss_newton), int(precision))


def solve_opts(npix_primary, kappa=0.3, damp_rel=1e-3, damp_abs=1e-12, pivot_min=1e-3, max_escalations=7,
               barrier_beta=1e-2, sh_floor=1e-3, scale_floor=0.1, opac_ftb=0.995, trust_pos=2.0, trust_rot=0.5,
               trust_scale=0.5, trust_sh=1.0, opac_eps=1e-6, step_frac=1.0, damp_sh=1e-3, precision=0, overlap=0,
               view_limit=0):
    """precision 0: plain form; 1: mixed form (BF16 matrix-core colour Grams, FP32 solves, FP64 for
    ill-conditioned position and rotation systems).  overlap 1: every kernel's steps times its overlap
    share (gsn_solve_opts.overlap_scale).  view_limit k > 0: only the first k view slots."""
    return CSolveOpts(damp_rel, damp_abs, pivot_min, max_escalations, barrier_beta, sh_floor, scale_floor,
                      opac_ftb, int(npix_primary), kappa, trust_pos, trust_rot, trust_scale, trust_sh, opac_eps,
                      step_frac, damp_sh, int(precision), int(overlap), int(view_limit))


def camera(c) -> CCamera:
    """synth.scenes.Camera -> C struct."""
    import numpy as np
    R = np.asarray(c.R, np.float32).reshape(-1)
    t = np.asarray(c.t, np.float32)
    return CCamera((ctypes.c_float * 9)(*R.tolist()), (ctypes.c_float * 3)(*t.tolist()), c.fx, c.fy, c.cx,
                   c.cy, c.width, c.height, c.znear)


def _ptr(t: torch.Tensor):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


class DeviceGaussians:
    """Kernel attributes as device tensors: pos [3,N], rot [4,N], scale [3,N], opac [N], sh [3,K,N] (f32)."""

    def __init__(self, pos, rot, scale, opac, sh, sh_degree):
        self.pos, self.rot, self.scale, self.opac, self.sh = pos, rot, scale, opac, sh
        self.sh_degree = int(sh_degree)

    @staticmethod
    def from_host(g, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).contiguous().to(device)  # noqa: E731
        return DeviceGaussians(f(g.pos), f(g.rot), f(g.scale), f(g.opac), f(g.sh), g.sh_degree)

    @property
    def n(self):
        return int(self.pos.shape[1])

    def clone(self):
        return DeviceGaussians(self.pos.clone(), self.rot.clone(), self.scale.clone(), self.opac.clone(),
                               self.sh.clone(), self.sh_degree)

    def c(self) -> CGaussians:
        return CGaussians(_ptr(self.pos), _ptr(self.rot), _ptr(self.scale), _ptr(self.opac), _ptr(self.sh),
                          self.n, self.sh_degree)

    def to_host(self):
        from synth.scenes import Gaussians
        return Gaussians(self.pos.cpu().numpy(), self.rot.cpu().numpy(), self.scale.cpu().numpy(),
                         self.opac.cpu().numpy(), self.sh.cpu().numpy(), self.sh_degree)


class Frame:
    def __init__(self, ctx: "Context"):
        self.ctx = ctx
        h = ctypes.c_void_p()
        ctx._check(lib().gsn_frame_create(ctx.h, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().gsn_frame_destroy(self.ctx.h, self.h)
            self.h = None

    def reserve(self, n, width, height, max_pairs):
        """gsn_frame_reserve: size every buffer once (max_pairs = 0 returns to growing mode)."""
        self.ctx._check(lib().gsn_frame_reserve(self.ctx.h, self.h, int(n), int(width), int(height),
                                                int(max_pairs)))

    def info(self):
        pairs, tx, ty = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self.ctx._check(lib().gsn_frame_info(self.ctx.h, self.h, ctypes.byref(pairs), ctypes.byref(tx),
                                             ctypes.byref(ty)))
        return pairs.value, tx.value, ty.value

    def lists(self, n, npix):
        """Copies of (ranges [tiles,2] u32, ids [pairs] u32, depth bits [n] u32, rect [4,n] i32, ncontrib [npix])."""
        pairs, tx, ty = self.info()
        dev = self.ctx.device
        ranges = torch.zeros(tx * ty * 2, dtype=torch.int32, device=dev)
        ids = torch.zeros(max(pairs, 1), dtype=torch.int32, device=dev)
        depth = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
        rect = torch.zeros(4 * max(n, 1), dtype=torch.int32, device=dev)
        nc = torch.zeros(npix, dtype=torch.int32, device=dev)
        self.ctx._check(lib().gsn_frame_lists(self.ctx.h, self.h, _ptr(ranges), _ptr(ids), _ptr(depth),
                                              _ptr(rect), _ptr(nc)))
        torch.cuda.synchronize(dev)
        return ranges.view(-1, 2), ids[:pairs], depth[:n], rect[:4 * n].view(4, n), nc

    def loss_maps(self, H, W):
        dL = torch.zeros(3, H, W, dtype=torch.float32, device=self.ctx.device)
        h = torch.zeros(3, H, W, dtype=torch.float32, device=self.ctx.device)
        self.ctx._check(lib().gsn_frame_loss_maps(self.ctx.h, self.h, _ptr(dL), _ptr(h)))
        return dL, h

    def records(self, n):
        """[12, n]: mx, my, q1, q2, cos, sin, sigma, colour (3), 0, 0 (see gsn_frame_records)."""
        out = torch.zeros(3 * 4 * max(n, 1), dtype=torch.float32, device=self.ctx.device)
        self.ctx._check(lib().gsn_frame_records(self.ctx.h, self.h, _ptr(out)))
        return out[:12 * n].view(3, n, 4).permute(0, 2, 1).reshape(12, n)

    def zstats(self, n):
        out = torch.zeros(GSN_NZ * max(n, 1), dtype=torch.float32, device=self.ctx.device)
        self.ctx._check(lib().gsn_frame_zstats(self.ctx.h, self.h, _ptr(out)))
        return out[:GSN_NZ * n].view(GSN_NZ, n)


class Context:
    def __init__(self, device=0, stream=None):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index if self.device.index is not None else 0
        stream = stream or torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = lib().gsn_create(ctypes.byref(h), idx, ctypes.c_void_p(stream.cuda_stream))
        if st != 0:
            raise GsnError(st, "gsn_create failed (no HIP device?)")
        self.h = h
        self.stream = stream

    def _check(self, st):
        if st != 0:
            raise GsnError(st, lib().gsn_last_error(self.h).decode())

    def close(self):
        if self.h:
            lib().gsn_destroy(self.h)
            self.h = None

    def frame(self) -> Frame:
        return Frame(self)

    def render(self, g: DeviceGaussians, cam: CCamera, ro: CRenderOpts, frame: Frame, rgb=None, T=None):
        cg = g.c()
        self._check(lib().gsn_render(self.h, ctypes.byref(cg), ctypes.byref(cam), ctypes.byref(ro), frame.h,
                                     _ptr(rgb), _ptr(T)))

    def accumulate_hessian(self, g, frame, target, lo: CLossOpts, view_slot, blocks: "Blocks", loss_out=None):
        cg = g.c()
        cb = blocks.c()
        self._check(lib().gsn_accumulate_hessian(self.h, ctypes.byref(cg), frame.h, _ptr(target),
                                                 ctypes.byref(lo), int(view_slot), ctypes.byref(cb),
                                                 _ptr(loss_out)))

    def accumulate_views(self, g, cams, frames, targets, ro: CRenderOpts, lo: CLossOpts, blocks: "Blocks",
                         loss_out=None, first_slot=0, add_shares=True):
        """Render + accumulate of several views (view i into slot first_slot + i) with their work
        overlapped on the library's streams; loss_out: float64 [n_views][2] on the device, or None.
        add_shares False: the views' shares of the summed rows stay in the frames (add_view_shares)."""
        n = len(cams)
        if not (len(frames) == len(targets) == n):
            raise ValueError("cams, frames and targets differ in length")
        if loss_out is not None and (loss_out.dtype != torch.float64 or not loss_out.is_contiguous()
                                     or loss_out.numel() < 2 * n):
            raise ValueError("loss_out must be a contiguous float64 tensor of at least [n_views][2]")
        cg, cb = g.c(), blocks.c()
        ccams = (CCamera * n)(*cams)
        hfr = (ctypes.c_void_p * n)(*[f.h.value for f in frames])
        htg = (ctypes.c_void_p * n)(*[t.data_ptr() for t in targets])
        self._check(lib().gsn_accumulate_views(self.h, ctypes.byref(cg), n, int(first_slot), ccams, hfr, htg,
                                               ctypes.byref(ro), ctypes.byref(lo), ctypes.byref(cb),
                                               _ptr(loss_out), int(bool(add_shares))))

    def add_view_shares(self, blocks: "Blocks", frames):
        """Adds the frames' shares of the summed rows to the blocks, in the order given."""
        cb = blocks.c()
        hfr = (ctypes.c_void_p * len(frames))(*[f.h.value for f in frames])
        self._check(lib().gsn_add_view_shares(self.h, ctypes.byref(cb), len(frames), hfr))

    def local_newton_solve(self, g, primary: CCamera, blocks: "Blocks", so: CSolveOpts, steps: "Steps"):
        cg, cb, cs = g.c(), blocks.c(), steps.c()
        self._check(lib().gsn_local_newton_solve(self.h, ctypes.byref(cg), ctypes.byref(primary),
                                                 ctypes.byref(cb), ctypes.byref(so), ctypes.byref(cs)))

    def local_newton_solve_noalloc(self, g, primary: CCamera, blocks: "Blocks", so: CSolveOpts, steps: "Steps"):
        """gsn_local_newton_solve_noalloc: the same solve with no device allocation."""
        cg, cb, cs = g.c(), blocks.c(), steps.c()
        self._check(lib().gsn_local_newton_solve_noalloc(self.h, ctypes.byref(cg), ctypes.byref(primary),
                                                         ctypes.byref(cb), ctypes.byref(so), ctypes.byref(cs)))

    def apply_step(self, g, steps: "Steps", so: CSolveOpts, group_mask=31, scale=None):
        """scale: None or a device float tensor [5, n] (per-group multipliers of the steps)."""
        cg, cs = g.c(), steps.c()
        self._check(lib().gsn_apply_step(self.h, ctypes.byref(cg), ctypes.byref(cs), ctypes.byref(so),
                                         _ptr(scale), int(group_mask)))

    def solve_apply(self, g, primary: CCamera, blocks: "Blocks", so: CSolveOpts, steps: "Steps", group_mask=31):
        """gsn_solve_apply: the solve and the update of the groups in group_mask in one launch."""
        cg, cb, cs = g.c(), blocks.c(), steps.c()
        self._check(lib().gsn_solve_apply(self.h, ctypes.byref(cg), ctypes.byref(primary), ctypes.byref(cb),
                                          ctypes.byref(so), ctypes.byref(cs), int(group_mask)))

    def first_order_step(self, g, blocks: "Blocks", so: CSolveOpts, lr, adam=True, step=1, state=None,
                         beta1=0.9, beta2=0.999, eps=1e-15, group_mask=31):
        """One gradient-descent (adam=False) or Adam step from the gradients in `blocks`.
        lr: five learning rates (position, rotation, scaling, opacity, colour); state: device
        float tensor [2, 10 + 3K, n] of moments, zeroed before step 1."""
        cg, cb = g.c(), blocks.c()
        fo = CFirstOrderOpts((ctypes.c_float * 5)(*[float(x) for x in lr]), beta1, beta2, eps, int(adam), int(step))
        self._check(lib().gsn_first_order_step(self.h, ctypes.byref(cg), ctypes.byref(cb), ctypes.byref(so),
                                               ctypes.byref(fo), _ptr(state), int(group_mask)))

    def _items(self, items):
        """items: list of (DeviceGaussians, CCamera, Blocks, CSolveOpts, Steps) -> C array (+ keep-alive)."""
        keep = []
        arr = (CSolveItem * len(items))()
        for i, (g, cam, blocks, so, steps) in enumerate(items):
            cg, cb, cs = g.c(), blocks.c(), steps.c()
            keep += [cg, cb, cs, cam, so]
            arr[i] = CSolveItem(ctypes.addressof(cg), ctypes.addressof(cam), ctypes.addressof(cb),
                                ctypes.addressof(so), ctypes.addressof(cs))
        return arr, keep

    def sh_gram(self, blocks: "Blocks", sh_degree, out):
        """out: device float [10, n]."""
        cb = blocks.c()
        self._check(lib().gsn_sh_gram(self.h, ctypes.byref(cb), int(sh_degree), _ptr(out)))

    def solve_batched(self, items):
        arr, keep = self._items(items)
        self._check(lib().gsn_solve_batched(self.h, arr, len(items)))

    def solve_tune(self, items):
        arr, keep = self._items(items)
        b, gr = ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().gsn_solve_tune(self.h, arr, len(items), ctypes.byref(b), ctypes.byref(gr)))
        return int(b.value), int(gr.value)

    def solve_graph(self, items) -> "SolveGraph":
        arr, keep = self._items(items)
        h = ctypes.c_void_p()
        self._check(lib().gsn_solve_graph_create(self.h, arr, len(items), ctypes.byref(h)))
        return SolveGraph(self, h)

    def step_features(self, g, primary: CCamera, blocks: "Blocks", so: CSolveOpts, feat, ok, resid=None):
        """feat: device float [17, n]; ok: device uint8 [n]; resid: device float [n] (the cached
        neighbouring-view residuals) or None."""
        cg, cb = g.c(), blocks.c()
        self._check(lib().gsn_step_features(self.h, ctypes.byref(cg), ctypes.byref(primary), ctypes.byref(cb),
                                            ctypes.byref(so), _ptr(resid), _ptr(feat), _ptr(ok)))

    def neighbour_residual(self, blocks: "Blocks", resid):
        """gsn_neighbour_residual: updates the cache resid (device float [n]) from full-rule blocks."""
        cb = blocks.c()
        self._check(lib().gsn_neighbour_residual(self.h, ctypes.byref(cb), _ptr(resid)))

    def step_labels(self, prim: "Steps", aug: "Steps", label, mask, ok=None, alpha=None, err=None):
        """label, mask: device float [5, n]; ok: device uint8 [n] feature status (or None); alpha: the
        network's scales [5, n] and err: device float64 [2] (+= sum mask |alpha - label|, sum mask), or None."""
        cp, ca = prim.c(), aug.c()
        self._check(lib().gsn_step_labels(self.h, ctypes.byref(cp), ctypes.byref(ca), _ptr(ok), _ptr(alpha),
                                          _ptr(label), _ptr(mask), _ptr(err)))

    def mlp_reset(self, mlp: "MLP"):
        self._check(lib().gsn_mlp_reset(self.h, ctypes.byref(mlp.cs)))

    def mlp_infer(self, mlp: "MLP", feat, ok, alpha, out_of_range=None):
        """out_of_range: device int32 [1] (+= kernels whose features left the trained range), or None."""
        n = int(ok.numel())
        self._check(lib().gsn_mlp_infer(self.h, ctypes.byref(mlp.cs), n, _ptr(feat), _ptr(ok), _ptr(alpha),
                                        _ptr(out_of_range)))

    def mlp_train_step(self, mlp: "MLP", feat, label, mask, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                       loss=None, grad=None):
        n = int(label.shape[1]) if label.dim() == 2 else 0
        a = CAdamOpts(lr, beta1, beta2, eps)
        self._check(lib().gsn_mlp_train_step(self.h, ctypes.byref(mlp.cs), n, _ptr(feat), _ptr(label), _ptr(mask),
                                             ctypes.byref(a), _ptr(loss), _ptr(grad)))

    STAGES = ("project", "sort", "raster_fwd", "loss", "raster_bwd", "chain", "solve", "apply")
    GROUPS4 = ("position", "rotation", "scaling", "opacity")
    COUNTERS = (("fwd_evals", "bwd_evals", "bwd_active", "pairs", "partials", "fwd_staged", "fp64_solves",
                 "bwd_staged")
                + tuple(f"escalated_{g}" for g in GROUPS4) + tuple(f"fallback_{g}" for g in GROUPS4)
                + tuple(f"clamped_{g}" for g in ("position", "rotation", "scaling", "colour"))
                + ("solved", "opacity_bound", "fwd_wave_steps", "bwd_wave_steps")
                + tuple(f"bwd_cycles_{p}" for p in ("stage", "scan", "walk", "sums")))

    def sync_status(self):
        """gsn_sync_status: (status code, {counter: value}, message); synchronises the stream and clears
        the counters.  The status is GSN_OK, GSN_E_NUMERIC or GSN_E_CAPACITY (not raised)."""
        import numpy as np
        out = np.zeros(len(STATS), np.int64)
        st = lib().gsn_sync_status(self.h, out.ctypes.data_as(ctypes.c_void_p))
        if st not in (0, GSN_E_NUMERIC, GSN_E_CAPACITY):
            self._check(st)
        return st, {k: int(out[i]) for i, k in enumerate(STATS)}, lib().gsn_last_error(self.h).decode()

    def capture(self, fn) -> "SolveGraph":
        """Records the library calls fn() makes on this context into a graph (gsn_capture_begin/end);
        Graph.launch() replays them on the context's stream."""
        self._check(lib().gsn_capture_begin(self.h))
        try:
            fn()
        finally:
            h = ctypes.c_void_p()
            st = lib().gsn_capture_end(self.h, ctypes.byref(h))
        self._check(st)
        return SolveGraph(self, h)

    def profile_enable(self, on=True, steps=False):
        """steps: also count the raster passes' wave steps (profiling level 2, slower rasters)."""
        self._check(lib().gsn_profile_enable(self.h, (2 if steps else 1) if on else 0))

    def profile_read(self):
        """{stage: (ms, launches)}, {counter: value}; synchronises the stream."""
        import numpy as np
        ms = np.zeros(len(self.STAGES), np.float64)
        nl = np.zeros(len(self.STAGES), np.int64)
        cnt = np.zeros(len(self.COUNTERS), np.int64)
        self._check(lib().gsn_profile_read(self.h, ms.ctypes.data_as(ctypes.c_void_p),
                                           nl.ctypes.data_as(ctypes.c_void_p), cnt.ctypes.data_as(ctypes.c_void_p)))
        return ({s: (float(ms[i]), int(nl[i])) for i, s in enumerate(self.STAGES)},
                {c: int(cnt[i]) for i, c in enumerate(self.COUNTERS)})

    def scene_center(self, g: DeviceGaussians, out):
        """out: device float64 tensor [3] (mean kernel position, Sec. 4.1)."""
        cg = g.c()
        self._check(lib().gsn_scene_center(self.h, ctypes.byref(cg), _ptr(out)))

    def blocks_zero(self, blocks: "Blocks"):
        cb = blocks.c()
        self._check(lib().gsn_blocks_zero(self.h, ctypes.byref(cb)))

    def downsample2x(self, src, W, H, dst):
        self._check(lib().gsn_downsample2x(self.h, _ptr(src), int(W), int(H), _ptr(dst)))


GSN_MLP_IN, GSN_MLP_PARAMS = 17, 741


class CMlp(ctypes.Structure):
    _fields_ = [("d_params", ctypes.c_void_p), ("d_m", ctypes.c_void_p), ("d_v", ctypes.c_void_p),
                ("d_half", ctypes.c_void_p), ("step", ctypes.c_int32)]


class CFirstOrderOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 5), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("adam", ctypes.c_int32), ("step", ctypes.c_int32)]


class CSolveItem(ctypes.Structure):
    _fields_ = [("g", ctypes.c_void_p), ("primary", ctypes.c_void_p), ("blocks", ctypes.c_void_p),
                ("opts", ctypes.c_void_p), ("steps", ctypes.c_void_p)]


class SolveGraph:
    """A captured batched solve or sequence of calls; launch() replays it on the context's stream."""

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def launch(self):
        self.ctx._check(lib().gsn_graph_launch(self.ctx.h, self.h))

    def close(self):
        if self.h is not None:
            lib().gsn_graph_destroy(self.ctx.h, self.h)
            self.h = None


class CAdamOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class MLP:
    """Step-scale network state as device tensors (FP32 master weights, Adam moments, FP16 copy)."""

    def __init__(self, params, device):
        import numpy as np
        p = np.asarray(params, np.float32).reshape(-1)
        if p.size != GSN_MLP_PARAMS:
            raise ValueError(f"expected {GSN_MLP_PARAMS} parameters")
        self.params = torch.tensor(p, device=device)
        self.m = torch.zeros(GSN_MLP_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros(GSN_MLP_PARAMS, dtype=torch.float32, device=device)
        self.half = torch.zeros(GSN_MLP_PARAMS, dtype=torch.float16, device=device)
        self.cs = CMlp(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(self.half), 0)

    @property
    def step(self):
        return int(self.cs.step)


class Blocks:
    def __init__(self, n, n_views, device):
        self.n, self.n_views = int(n), int(n_views)
        nf = lib().gsn_blocks_floats(self.n, self.n_views)
        self.data = torch.zeros(max(nf, 1), dtype=torch.float32, device=device)

    def c(self):
        return CBlocks(_ptr(self.data), self.n, self.n_views)

    def view(self):
        """Rows [30 + 10 V + 1, n] (see gsn.h: base rows, V view slots, the overlap numerator)."""
        return self.data[:(GSN_BLK_BASE + GSN_BLK_VIEW * self.n_views + 1) * self.n].view(-1, self.n)


class Steps:
    def __init__(self, n, sh_degree, device):
        self.n, self.sh_degree = int(n), int(sh_degree)
        nf = lib().gsn_steps_floats(self.n, self.sh_degree)
        self.data = torch.zeros(max(nf, 1), dtype=torch.float32, device=device)
        self.flags = torch.zeros(5 * max(self.n, 1), dtype=torch.int32, device=device)

    def c(self):
        return CSteps(_ptr(self.data), _ptr(self.flags), self.n, self.sh_degree)

    def view(self):
        K = (self.sh_degree + 1) ** 2
        return self.data[:(GSN_STEP_BASE + 3 * K) * self.n].view(-1, self.n), self.flags[:5 * self.n].view(5, self.n)


def camera_half(cam: CCamera) -> CCamera:
    """Camera of the half-resolution secondary target of `cam` (gsn_camera_half)."""
    out = CCamera()
    st = lib().gsn_camera_half(ctypes.byref(cam), ctypes.byref(out))
    if st != 0:
        raise GsnError(st, "gsn_camera_half: image smaller than 2x2")
    return out


def camera_knn(centers, scene_center, k=3):
    import numpy as np
    c = np.ascontiguousarray(centers, np.float64)
    sc = np.ascontiguousarray(scene_center, np.float64)
    out = np.zeros((c.shape[0], k), np.int32)
    st = lib().gsn_camera_knn(c.ctypes.data_as(ctypes.c_void_p), c.shape[0], sc.ctypes.data_as(ctypes.c_void_p),
                              k, out.ctypes.data_as(ctypes.c_void_p))
    if st != 0:
        raise GsnError(st, "gsn_camera_knn: k must be in 1..ncam-1")
    return out
