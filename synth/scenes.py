"""Seeded scene and camera generators (inputs only).

Layout conventions used everywhere in this repository:

* Gaussians are structure-of-arrays, float32:
  ``pos[3][N]``, ``rot[4][N]`` (quaternion w, x, y, z), ``scale[3][N]`` (linear
  axis lengths s > 0), ``opac[N]`` (opacity in (0, 1)), ``sh[3][K][N]`` with
  K = (degree + 1)^2 coefficients per colour channel.
* Cameras are world-to-camera rigid transforms with OpenCV axes (x right,
  y down, z forward), pinhole intrinsics fx, fy, cx, cy, and pixel centres at
  integer coordinates, so cx = (W - 1) / 2.

The synthetic workloads stand in for the paper's photographic datasets
(Mip-NeRF360, Tanks&Temples, DeepBlending, Sec. 5), which are not used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Constant of the degree-0 real spherical harmonic, 1 / (2 sqrt(pi)).  The
# generator needs it only to express an RGB draw as a DC coefficient.
Y00 = 0.5 / math.sqrt(math.pi)


def sh_coeffs_per_channel(degree: int) -> int:
    return (degree + 1) ** 2


@dataclass
class Gaussians:
    pos: np.ndarray    # [3][N] f32
    rot: np.ndarray    # [4][N] f32 (w, x, y, z)
    scale: np.ndarray  # [3][N] f32 linear
    opac: np.ndarray   # [N] f32
    sh: np.ndarray     # [3][K][N] f32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    def copy(self) -> "Gaussians":
        return Gaussians(self.pos.copy(), self.rot.copy(), self.scale.copy(),
                         self.opac.copy(), self.sh.copy(), self.sh_degree)

    def subset(self, idx) -> "Gaussians":
        idx = np.asarray(idx)
        return Gaussians(np.ascontiguousarray(self.pos[:, idx]),
                         np.ascontiguousarray(self.rot[:, idx]),
                         np.ascontiguousarray(self.scale[:, idx]),
                         np.ascontiguousarray(self.opac[idx]),
                         np.ascontiguousarray(self.sh[:, :, idx]), self.sh_degree)


@dataclass
class Camera:
    R: np.ndarray          # [3][3] f32, world -> camera rotation
    t: np.ndarray          # [3] f32, world -> camera translation
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def center(self) -> np.ndarray:
        """Camera centre in world coordinates, o = -R^T t (float64)."""
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


def pinhole_intrinsics(width: int, height: int, fov_x_deg: float):
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return (float(np.float32(fx)), float(np.float32(fx)),
            float(np.float32((width - 1) / 2.0)), float(np.float32((height - 1) / 2.0)))


def look_at_camera(eye, target, up, width, height, fov_x_deg=60.0, znear=0.2) -> Camera:
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(float(f @ up)) > 0.99 * np.linalg.norm(up):
        up = np.array([0.0, 1.0, 0.0]) if abs(f[1]) < 0.99 else np.array([1.0, 0.0, 0.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    fx, fy, cx, cy = pinhole_intrinsics(width, height, fov_x_deg)
    return Camera(R, t, fx, fy, cx, cy, width, height, znear)


def fibonacci_cameras(n, radius, width, height, fov_x_deg=60.0):
    """n cameras on a Fibonacci lattice of the given radius, looking at the origin, up = +z."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    cams = []
    for i in range(n):
        z = 1.0 - (2.0 * i + 1.0) / n
        r = math.sqrt(max(0.0, 1.0 - z * z))
        phi = golden * i
        eye = radius * np.array([r * math.cos(phi), r * math.sin(phi), z])
        cams.append(look_at_camera(eye, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), width, height, fov_x_deg))
    return cams


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _random_quaternions(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _uniform_sphere(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _sh_block(rng, n, degree):
    K = sh_coeffs_per_channel(degree)
    sh = np.zeros((3, K, n), np.float64)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    sh[:, 0, :] = rgb / Y00
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.1, size=(3, K - 1, n))
    return sh


def surface_scene(n, seed, sh_degree=3, n_surfaces=20):
    """Kernels on random spheres and planes, anisotropic scales, random rotations."""
    rng = np.random.default_rng(seed)
    surfs = []
    for _ in range(n_surfaces):
        if rng.uniform() < 0.5:
            c = rng.uniform(-0.6, 0.6, 3)
            r = rng.uniform(0.15, 0.4)
            surfs.append(("sphere", c, r, 4.0 * math.pi * r * r))
        else:
            c = rng.uniform(-0.6, 0.6, 3)
            nrm = _uniform_sphere(rng, 1)[0]
            a, b = rng.uniform(0.2, 0.6, 2)
            surfs.append(("plane", c, (nrm, a, b), 4.0 * a * b))
    areas = np.array([s[3] for s in surfs])
    share = n * areas / areas.sum()
    counts = np.floor(share).astype(np.int64)
    rem = n - int(counts.sum())
    order = np.argsort(-(share - counts), kind="stable")
    counts[order[:rem]] += 1
    pts = []
    for (kind, c, geo, _), m in zip(surfs, counts):
        if m == 0:
            continue
        if kind == "sphere":
            pts.append(c + geo * _uniform_sphere(rng, m))
        else:
            nrm, a, b = geo
            ref = np.array([0.0, 0.0, 1.0]) if abs(nrm[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
            e1 = np.cross(nrm, ref)
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(nrm, e1)
            uv = rng.uniform(-1.0, 1.0, (m, 2))
            pts.append(c + uv[:, :1] * a * e1 + uv[:, 1:] * b * e2)
    pos = np.concatenate(pts, 0).T
    log_s = rng.normal(-4.0, 0.5, (3, n))
    rot = _random_quaternions(rng, n)
    opac = _sigmoid(rng.standard_normal(n))
    sh = _sh_block(rng, n, sh_degree)
    return Gaussians(pos.astype(np.float32), rot.astype(np.float32),
                     np.exp(log_s).astype(np.float32), opac.astype(np.float32),
                     sh.astype(np.float32), sh_degree)


def cube_scene(n, seed):
    """Isotropic kernels uniform in [-1,1]^3, identity rotation, SH degree 0."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-1.0, 1.0, (3, n))
    log_s = rng.normal(-3.0, 0.3, n)
    scale = np.repeat(np.exp(log_s)[None, :], 3, 0)
    rot = np.zeros((4, n))
    rot[0] = 1.0
    opac = _sigmoid(rng.standard_normal(n))
    sh = _sh_block(rng, n, 0)
    return Gaussians(pos.astype(np.float32), rot.astype(np.float32), scale.astype(np.float32),
                     opac.astype(np.float32), sh.astype(np.float32), 0)


def perturb(g: Gaussians, seed, pos_sigma=0.05, log_scale_sigma=0.2) -> Gaussians:
    """Starting state: position + N(0, pos_sigma) per coordinate, log-scale + N(0, log_scale_sigma) per axis."""
    rng = np.random.default_rng(seed)
    out = g.copy()
    out.pos = (g.pos.astype(np.float64) + rng.normal(0.0, pos_sigma, g.pos.shape)).astype(np.float32)
    out.scale = (g.scale.astype(np.float64)
                 * np.exp(rng.normal(0.0, log_scale_sigma, g.scale.shape))).astype(np.float32)
    return out


def deep_list_scene(seed: int, n: int = 4000):
    """A single 16x16 tile whose list is n entries deep: n small, faint kernels (opacity 0.04-0.08,
    scale about 0.7 px) spread over a 16x16 view at distance 4, so that every pixel keeps
    compositing far down the depth-sorted list.  Returns (ground truth, perturbed start, camera)."""
    rng = np.random.default_rng(seed)
    pos = np.zeros((3, n))
    pos[0] = rng.uniform(-2.4, 2.4, n)
    pos[1] = rng.uniform(-2.4, 2.4, n)
    pos[2] = rng.uniform(-0.5, 0.5, n)
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0)
    scale = np.exp(rng.normal(math.log(0.2), 0.2, (3, n)))
    opac = rng.uniform(0.04, 0.08, n)
    sh = rng.uniform(0.1, 0.9, (3, 1, n)) / Y00
    gt = Gaussians(pos.astype(np.float32), q.astype(np.float32), scale.astype(np.float32),
                   opac.astype(np.float32), sh.astype(np.float32), 0)
    cam = look_at_camera((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), (0.0, -1.0, 0.0), 16, 16, 60.0)
    return gt, perturb(gt, seed + 1, pos_sigma=0.02), cam


@dataclass
class Config:
    name: str
    n: int
    sh_degree: int
    n_views: int
    width: int
    height: int
    seed: int
    n_secondary: int
    epochs: int
    gt: Gaussians = field(repr=False, default=None)
    init: Gaussians = field(repr=False, default=None)
    cams: list = field(repr=False, default=None)


CONFIGS = {
    "c0": dict(n=256, sh_degree=0, n_views=1, width=64, height=64, seed=0, n_secondary=0, epochs=1),
    "c1": dict(n=100_000, sh_degree=3, n_views=50, width=1024, height=768, seed=1000,
               n_secondary=3, epochs=10),
    "c2": dict(n=1_000_000, sh_degree=3, n_views=150, width=1920, height=1080, seed=2000,
               n_secondary=3, epochs=1),
    "c4": dict(n=3_000_000, sh_degree=3, n_views=300, width=1920, height=1080, seed=4000,
               n_secondary=3, epochs=1),
}
C3_SIZES = (20_000, 50_000, 100_000, 200_000, 300_000, 400_000, 600_000, 800_000)


def make_config(name: str, n: int | None = None, width: int | None = None,
                height: int | None = None, n_views: int | None = None) -> Config:
    """Build a named workload.  Optional overrides shrink it for tests."""
    if name.startswith("c3_"):
        i = int(name[3:])
        spec = dict(n=C3_SIZES[i], sh_degree=3, n_views=32, width=1280, height=720,
                    seed=3000 + i, n_secondary=3, epochs=1)
    else:
        spec = dict(CONFIGS[name])
    if n is not None:
        spec["n"] = n
    if width is not None:
        spec["width"] = width
    if height is not None:
        spec["height"] = height
    if n_views is not None:
        spec["n_views"] = n_views
    cfg = Config(name=name, **spec)
    if name == "c0":
        cfg.gt = cube_scene(cfg.n, cfg.seed)
        cfg.init = perturb(cfg.gt, cfg.seed + 1)
        fx, fy, cx, cy = pinhole_intrinsics(cfg.width, cfg.height, 60.0)
        R = np.eye(3, dtype=np.float32)
        t = np.array([0.0, 0.0, 4.0], np.float32)
        cfg.cams = [Camera(R, t, fx, fy, cx, cy, cfg.width, cfg.height)]
    else:
        cfg.gt = surface_scene(cfg.n, cfg.seed, cfg.sh_degree)
        cfg.init = perturb(cfg.gt, cfg.seed + 1)
        cfg.cams = fibonacci_cameras(cfg.n_views, 4.0, cfg.width, cfg.height)
    return cfg


def view_order(n_views: int, epoch: int) -> np.ndarray:
    """Seeded per-epoch permutation of the training views (seed 7 + epoch)."""
    return np.random.default_rng(7 + epoch).permutation(n_views)
