"""Seeded synthetic inputs: Gaussian maps, camera rigs, target images, LiDAR depth.

This module is the only code shared by the HIP path, its tests, the benchmark and the
oracle's tests.  It produces *inputs* only and holds none of the rasteriser's arithmetic
(no projection of Gaussians, no compositing, no loss).  The LiDAR simulator casts rays
against the analytic orchard geometry (tree cylinders and a ground plane); it never looks
at the Gaussians.

The paper evaluates on private apple and pear orchard recordings with a three-camera rig
and a 32-beam LiDAR (Sec. IV and Fig. 2).  Those recordings are not available, so the
"orchard rows" below stand in for them: canopy clusters in vertical cylinders on parallel
rows, plus a ground plane of flat Gaussians, seen by a rig of pinhole cameras that drives
along the alley between two rows.

Conventions shared by every consumer:
  * world frame z-up; camera frame x right, y down, z forward (optical axis);
  * a camera stores the world->camera rotation R (3x3, row-major) and translation t,
    so a world point p maps to R p + t;
  * quaternions are (w, x, y, z) and need not be normalised;
  * SH coefficients are stored (N, K, 3) with K = (deg+1)^2, l-major, m = -l..l;
  * all float arrays are float32 (the precision the GPU consumes); the oracle upcasts the
    very same values to float64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# The degree-0 real spherical harmonic is the constant 1/(2 sqrt(pi)); the generator uses
# it only to store a chosen base colour as a DC coefficient.
_Y00 = 0.5 / math.sqrt(math.pi)

ROW_Y = (-10.0, -6.0, -2.0, 2.0, 6.0, 10.0)  # row centre lines, 4 m apart
TREE_SPACING = 1.5
TREE_RADIUS = 1.0
TREE_HEIGHT = 3.0


@dataclass
class Camera:
    R: np.ndarray          # (3, 3) float32, world -> camera
    t: np.ndarray          # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    g_begin: int = 0       # Gaussians [g_begin, g_end) are visible to this view
    g_end: int = -1

    def center(self) -> np.ndarray:
        """Camera centre in world coordinates (float64)."""
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclass
class Scene:
    means: np.ndarray            # (N, 3) float32
    log_scales: np.ndarray       # (N, 3) float32
    quats: np.ndarray            # (N, 4) float32, wxyz
    opacity_logits: np.ndarray   # (N,) float32
    sh: np.ndarray               # (N, K, 3) float32
    sh_degree: int
    cameras: list = field(default_factory=list)
    gt_rgb: list = field(default_factory=list)      # per view (3, H, W) float32
    lidar: list = field(default_factory=list)       # per view dict(pix, depth, sigma)
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cameras))

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                     self.opacity_logits.copy(), self.sh.copy(), self.sh_degree,
                     [Camera(c.R.copy(), c.t.copy(), c.fx, c.fy, c.cx, c.cy, c.width,
                             c.height, c.g_begin, c.g_end) for c in self.cameras],
                     [g.copy() for g in self.gt_rgb],
                     [{k: v.copy() for k, v in d.items()} for d in self.lidar], self.name)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _random_unit_quats(rng, n):
    q = rng.normal(size=(n, 4))
    return q / np.linalg.norm(q, axis=1, keepdims=True)


def _dc_from_rgb(rgb, degree, rng=None, rest_std=0.0):
    k = (degree + 1) ** 2
    sh = np.zeros((rgb.shape[0], k, 3))
    sh[:, 0, :] = (rgb - 0.5) / _Y00
    if k > 1 and rest_std > 0:
        sh[:, 1:, :] = rng.normal(0.0, rest_std, size=(rgb.shape[0], k - 1, 3))
    return sh


def look_camera(center, yaw_deg, width, height, f, pitch_deg=0.0):
    """Pinhole camera at `center` looking horizontally along azimuth `yaw_deg` (world z-up).

    Rows of R are the camera axes (right, down, forward) expressed in world coordinates.
    """
    yaw = math.radians(yaw_deg)
    pitch = math.radians(pitch_deg)
    fwd = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    c = np.asarray(center, dtype=np.float64)
    t = -R @ c
    return Camera(_f32(R), _f32(t), float(f), float(f), width / 2.0, height / 2.0, width, height)


# ----------------------------------------------------------------------------- config 1
def tiny_scene(seed: int = 2511, n: int = 2000, width: int = 128, height: int = 96) -> Scene:
    """2,000 Gaussians uniform in a 4 m cube centred 4 m in front of one 128x96 pinhole
    camera (fx = fy = 110, cx = 64, cy = 48, identity pose); log-scales N(-3, 0.3), random
    unit quaternions, opacity logits N(0, 1), RGB uniform [0, 1] stored as SH degree 0.
    The target image is uniform [0, 1] noise drawn with seed + 100."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-2.0, 2.0, size=(n, 3)) + np.array([0.0, 0.0, 4.0])
    log_scales = rng.normal(-3.0, 0.3, size=(n, 3))
    quats = _random_unit_quats(rng, n)
    logits = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    sh = _dc_from_rgb(rgb, 0)
    f = 110.0 * width / 128.0
    cam = Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), f, f, width / 2.0,
                 height / 2.0, width, height, 0, n)
    trng = np.random.default_rng(seed + 100)
    gt = trng.uniform(0.0, 1.0, size=(3, height, width))
    return Scene(_f32(means), _f32(log_scales), _f32(quats), _f32(logits), _f32(sh), 0,
                 [cam], [_f32(gt)], [empty_lidar()], name="tiny")


def empty_lidar():
    return {"pix": np.zeros(0, np.int32), "depth": np.zeros(0, np.float32),
            "sigma": np.zeros(0, np.float32)}


# ----------------------------------------------------------------------------- orchard
def orchard_gaussians(rng, n, sh_degree=3, x_range=(-30.0, 30.0), canopy_frac=0.85,
                      canopy_log_scale=(-3.0, 0.3), origin=(0.0, 0.0)):
    """Orchard-row Gaussian map: canopy clusters in vertical cylinders (r = 1 m, h = 3 m)
    centred on rows 4 m apart, trees every 1.5 m, plus 15 % flat ground Gaussians."""
    ox, oy = origin
    n_canopy = int(round(n * canopy_frac))
    n_ground = n - n_canopy
    tree_x = np.arange(x_range[0], x_range[1] + 1e-9, TREE_SPACING)
    trees = np.array([(x, y) for y in ROW_Y for x in tree_x])
    pick = rng.integers(0, len(trees), size=n_canopy)
    r = TREE_RADIUS * np.sqrt(rng.uniform(0, 1, n_canopy))
    th = rng.uniform(0, 2 * math.pi, n_canopy)
    canopy = np.stack([trees[pick, 0] + r * np.cos(th), trees[pick, 1] + r * np.sin(th),
                       rng.uniform(0.0, TREE_HEIGHT, n_canopy)], axis=1)
    c_ls = rng.normal(canopy_log_scale[0], canopy_log_scale[1], size=(n_canopy, 3))
    c_q = _random_unit_quats(rng, n_canopy)
    c_rgb = np.clip(np.array([0.22, 0.45, 0.15]) + rng.normal(0, 0.08, (n_canopy, 3)), 0, 1)

    gx0, gx1 = x_range[0] - 2.0, x_range[1] + 2.0
    ground = np.stack([rng.uniform(gx0, gx1, n_ground), rng.uniform(-14.0, 14.0, n_ground),
                       np.zeros(n_ground)], axis=1)
    g_ls = np.array([-2.5, -2.5, -5.3]) + rng.normal(0, 0.2, (n_ground, 3))
    yaw = rng.uniform(0, 2 * math.pi, n_ground)
    g_q = np.stack([np.cos(yaw / 2), np.zeros(n_ground), np.zeros(n_ground), np.sin(yaw / 2)], 1)
    g_rgb = np.clip(np.array([0.42, 0.33, 0.22]) + rng.normal(0, 0.06, (n_ground, 3)), 0, 1)

    means = np.concatenate([canopy, ground]) + np.array([ox, oy, 0.0])
    log_scales = np.concatenate([c_ls, g_ls])
    quats = np.concatenate([c_q, g_q])
    logits = rng.normal(0.0, 1.0, size=n)
    rgb = np.concatenate([c_rgb, g_rgb])
    sh = _dc_from_rgb(rgb, sh_degree, rng, rest_std=0.02)
    perm = rng.permutation(n)  # interleave canopy and ground in memory
    return (_f32(means[perm]), _f32(log_scales[perm]), _f32(quats[perm]), _f32(logits[perm]),
            _f32(sh[perm]))


def rig_cameras(rig_center, yaws, width, height, f, baseline=0.15):
    cams = []
    for yaw in yaws:
        y = math.radians(yaw)
        fwd = np.array([math.cos(y), math.sin(y), 0.0])
        cams.append(look_camera(np.asarray(rig_center) + baseline * fwd, yaw, width, height, f))
    return cams


def _ray_cast_orchard(origins, dirs, x_range=(-30.0, 30.0), origin=(0.0, 0.0)):
    """Distance along unit rays to the first hit of the analytic orchard (tree cylinders
    of radius 1 m and height 3 m, and the ground plane z = 0); inf where nothing is hit."""
    ox, oy = origin
    best = np.full(len(dirs), np.inf)
    dz = dirs[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = np.where(dz < -1e-9, -origins[:, 2] / dz, np.inf)
    best = np.minimum(best, np.where(tg > 0, tg, np.inf))
    tree_x = np.arange(x_range[0], x_range[1] + 1e-9, TREE_SPACING) + ox
    a = dirs[:, 0] ** 2 + dirs[:, 1] ** 2
    for ry in ROW_Y:
        for tx in tree_x:
            px = origins[:, 0] - tx
            py = origins[:, 1] - (ry + oy)
            b = 2 * (px * dirs[:, 0] + py * dirs[:, 1])
            c = px * px + py * py - TREE_RADIUS ** 2
            disc = b * b - 4 * a * c
            ok = (disc >= 0) & (a > 1e-12)
            sq = np.sqrt(np.where(ok, disc, 0.0))
            t0 = np.where(ok, (-b - sq) / (2 * np.where(a > 1e-12, a, 1.0)), np.inf)
            t0 = np.where(t0 > 1e-6, t0, np.inf)
            zh = origins[:, 2] + t0 * dz
            t0 = np.where((zh >= 0) & (zh <= TREE_HEIGHT), t0, np.inf)
            best = np.minimum(best, t0)
    return best


def simulate_lidar(cam: Camera, rng, target_frac=0.05, n_beams=64, elev_deg=22.5,
                   max_range=80.0, rel_noise=0.02, x_range=(-30.0, 30.0), origin=(0.0, 0.0)):
    """Sparse LiDAR depth targets for one camera.

    Beams of a `n_beams`-line scanner spanning +-`elev_deg` of elevation pass through the
    image on near-horizontal scan lines; along each visible line pixels are taken with a
    fixed azimuth stride chosen so that about `target_frac` of the image is covered before
    misses (sky) are removed.  Each kept pixel's ray is cast against the analytic orchard;
    the target depth is the camera-frame z of the hit with 2 % multiplicative noise, and
    sigma = 0.02 * true depth (the configuration's fixed-variance model).
    """
    W, H = cam.width, cam.height
    elev = np.linspace(-elev_deg, elev_deg, n_beams)
    rows = np.round(cam.cy - cam.fy * np.tan(np.radians(elev)) - 0.5).astype(np.int64)
    rows = np.unique(rows[(rows >= 0) & (rows < H)])
    if len(rows) == 0:
        return empty_lidar()
    n_cols = int(min(W, max(1, round(target_frac * W * H / len(rows)))))
    step = W / n_cols
    cols = np.unique(np.floor(np.arange(n_cols) * step + rng.uniform(0, step)).astype(np.int64))
    cols = cols[cols < W]
    py, px = np.meshgrid(rows, cols, indexing="ij")
    px = px.ravel()
    py = py.ravel()
    d_cam = np.stack([(px + 0.5 - cam.cx) / cam.fx, (py + 0.5 - cam.cy) / cam.fy,
                      np.ones_like(px, dtype=np.float64)], axis=1)
    R = cam.R.astype(np.float64)
    d_world = d_cam @ R  # R^T d for each row
    norm = np.linalg.norm(d_world, axis=1, keepdims=True)
    d_unit = d_world / norm
    c = cam.center()
    dist = _ray_cast_orchard(np.broadcast_to(c, d_unit.shape).copy(), d_unit, x_range, origin)
    hit = np.isfinite(dist) & (dist < max_range)
    z_true = dist[hit] / norm[hit, 0]  # camera-frame depth of the hit point
    pix = (py[hit] * W + px[hit]).astype(np.int32)
    depth = z_true * (1.0 + rel_noise * rng.normal(size=z_true.shape))
    sigma = 0.02 * z_true
    order = np.argsort(pix, kind="stable")
    return {"pix": pix[order], "depth": _f32(depth[order]), "sigma": _f32(sigma[order])}


def procedural_image(width, height, rng):
    """Smooth colour field plus noise, values in [0, 1]: a stand-in target image."""
    yy, xx = np.mgrid[0:height, 0:width]
    img = np.empty((3, height, width))
    for ch in range(3):
        a, b, p = rng.uniform(0.5, 3.0), rng.uniform(0.5, 3.0), rng.uniform(0, 2 * math.pi)
        img[ch] = 0.5 + 0.3 * np.sin(a * 2 * math.pi * xx / width + p) * np.cos(b * 2 * math.pi * yy / height)
    img += rng.normal(0, 0.05, img.shape)
    return _f32(np.clip(img, 0, 1))


def orchard_scene(seed: int, n: int, yaws, width: int, height: int, f: float,
                  rig_center=(0.0, 0.0, 1.2), sh_degree: int = 3, with_targets: bool = True,
                  name: str = "") -> Scene:
    rng = np.random.default_rng(seed)
    means, ls, q, lo, sh = orchard_gaussians(rng, n, sh_degree)
    cams = rig_cameras(rig_center, yaws, width, height, f)
    for c in cams:
        c.g_begin, c.g_end = 0, n
    scene = Scene(means, ls, q, lo, sh, sh_degree, cams, name=name)
    if with_targets:
        for c in cams:
            scene.gt_rgb.append(procedural_image(c.width, c.height, rng))
            scene.lidar.append(simulate_lidar(c, rng))
    return scene


def single_view_scene(seed: int = 2512, n: int = 300_000) -> Scene:
    """One 960x600 camera (f = 825, same horizontal FOV as the tiny case) in the alley
    y = 0, 1.2 m high, looking along the rows; 300k orchard Gaussians, SH degree 3."""
    return orchard_scene(seed, n, [0.0], 960, 600, 825.0, name="single_view_300k")


def multi_view_scene(seed: int = 2513, n: int = 1_000_000, width: int = 1280,
                     height: int = 800) -> Scene:
    """Four-camera rig (yaw 0, +60, -60, 180 deg; 0.3 m front/back baseline) at
    1280x800 (f = 1100) over 1M orchard Gaussians, SH degree 3."""
    f = 1100.0 * width / 1280.0
    return orchard_scene(seed, n, [0.0, 60.0, -60.0, 180.0], width, height, f,
                         name=f"multi_view_{n // 1000}k")


def refinement_scene(seed: int = 2515, n: int = 2_000_000) -> Scene:
    """Four-view 1280x800 rig over 2M orchard Gaussians (the pose + map refinement case)."""
    return orchard_scene(seed, n, [0.0, 60.0, -60.0, 180.0], 1280, 800, 1100.0,
                         name="refine_2M")


SUBMAP_SIZES = (50_000, 100_000, 150_000, 250_000, 400_000, 500_000, 650_000, 800_000)
SUBMAP_RES = ((640, 400), (800, 500), (960, 600), (1120, 700), (1280, 800))


def submap_scene(seed: int = 2514, sizes=SUBMAP_SIZES, with_targets: bool = True,
                 spacing: float = 0.0, name: str = "submaps_2.9M") -> Scene:
    """Eight independent orchard patches of uneven size, concatenated into one Gaussian
    array; each patch is seen by 1-4 views (seeded) whose Gaussian range is that patch.
    Patch k sits at x = spacing * k of one shared world frame: spacing 0 gives every patch
    its own submap frame (origin at the patch), spacing 200 m lays the patches out along one
    global map, 1.4 km end to end (float32 world coordinates there are spaced 1.2e-4 m)."""
    rng = np.random.default_rng(seed)
    vrng = np.random.default_rng(seed + 200)
    parts, cams = [], []
    g0 = 0
    for k, n in enumerate(sizes):
        # each patch is a 12 m slice of orchard
        ox = spacing * k
        m, ls, q, lo, sh = orchard_gaussians(rng, n, 3, x_range=(-6.0, 6.0), origin=(ox, 0.0))
        parts.append((m, ls, q, lo, sh))
        n_views = int(vrng.integers(1, 5))
        yaws = vrng.choice([0.0, 60.0, -60.0, 180.0], size=n_views, replace=False)
        w, h = SUBMAP_RES[int(vrng.integers(0, len(SUBMAP_RES)))]
        for c in rig_cameras((ox - 3.0, 0.0, 1.2), yaws, w, h, 110.0 / 128.0 * w):
            c.g_begin, c.g_end = g0, g0 + n
            cams.append(c)
        g0 += n
    cat = [np.concatenate([p[j] for p in parts]) for j in range(5)]
    scene = Scene(_f32(cat[0]), _f32(cat[1]), _f32(cat[2]), _f32(cat[3]), _f32(cat[4]), 3,
                  cams, name=name)
    if with_targets:
        offsets = np.cumsum([0] + list(sizes))
        for c in cams:
            k = int(np.searchsorted(offsets, c.g_begin, side="right") - 1)
            scene.gt_rgb.append(procedural_image(c.width, c.height, rng))
            scene.lidar.append(simulate_lidar(c, rng, x_range=(-6.0, 6.0), origin=(spacing * k, 0.0)))
    return scene


def submap_far_scene(seed: int = 2514) -> Scene:
    """The sub-map workload with the eight patches 200 m apart in one global frame."""
    return submap_scene(seed, spacing=200.0, name="submaps_far_2.9M")


def perturb(scene: Scene, seed: int, mean_std=0.01, rho_std=0.02, phi_deg=0.5) -> Scene:
    """A copy with Gaussian means jittered (1 cm) and every camera pose perturbed by a
    random rotation (0.5 deg std per axis, about the camera centre) and translation (2 cm)."""
    rng = np.random.default_rng(seed)
    s = scene.copy()
    s.means = _f32(s.means + rng.normal(0, mean_std, s.means.shape))
    for c in s.cameras:
        ax = rng.normal(0, math.radians(phi_deg), 3)
        th = np.linalg.norm(ax)
        K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        dR = np.eye(3) + (math.sin(th) / th if th > 0 else 1.0) * K + \
            ((1 - math.cos(th)) / th ** 2 if th > 0 else 0.5) * K @ K
        R = dR @ c.R.astype(np.float64)
        t = dR @ c.t.astype(np.float64) + rng.normal(0, rho_std, 3)
        c.R, c.t = _f32(R), _f32(t)
    return s


CONFIGS = {
    "tiny": tiny_scene,
    "single_view": single_view_scene,
    "multi_view": multi_view_scene,
    "submaps": submap_scene,
    "submaps_far": submap_far_scene,
    "refine": refinement_scene,
}
