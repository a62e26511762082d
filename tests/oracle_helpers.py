"""Small scene builders for the oracle pin tests (inputs only, no rasteriser arithmetic)."""
import math

import numpy as np

from paper_2510_26358_amd.scenes import Camera, Scene, empty_lidar


def camera(R=None, t=None, f=100.0, width=32, height=24, fy=None, cx=None, cy=None, dtype=np.float64):
    R = np.eye(3) if R is None else np.asarray(R)
    t = np.zeros(3) if t is None else np.asarray(t)
    return Camera(R.astype(dtype), t.astype(dtype), float(f), float(fy if fy is not None else f),
                  width / 2.0 if cx is None else cx, height / 2.0 if cy is None else cy,
                  width, height, 0, -1)


def scene(means, log_scales=None, quats=None, logits=None, rgb=None, sh=None, cams=None,
          sh_degree=0, gt=None, lidar=None, dtype=np.float64):
    means = np.asarray(means, np.float64).reshape(-1, 3)
    n = len(means)
    log_scales = np.full((n, 3), -2.0) if log_scales is None else np.asarray(log_scales).reshape(n, 3)
    quats = np.tile([1.0, 0, 0, 0], (n, 1)) if quats is None else np.asarray(quats).reshape(n, 4)
    logits = np.zeros(n) if logits is None else np.asarray(logits, np.float64).reshape(n)
    if sh is None:
        k = (sh_degree + 1) ** 2
        sh = np.zeros((n, k, 3))
        if rgb is not None:
            sh[:, 0, :] = (np.asarray(rgb).reshape(n, 3) - 0.5) / (0.5 / math.sqrt(math.pi))
    cams = cams or [camera()]
    for c in cams:
        c.g_begin, c.g_end = 0, n
    sc = Scene(means.astype(dtype), log_scales.astype(dtype), quats.astype(dtype),
               logits.astype(dtype), np.asarray(sh).astype(dtype), sh_degree, cams)
    sc.gt_rgb = gt if gt is not None else [np.zeros((3, c.height, c.width)) for c in cams]
    sc.lidar = lidar if lidar is not None else [empty_lidar() for _ in cams]
    return sc


def logit(o):
    return math.log(o / (1 - o))


def random_scene(seed, n=60, width=32, height=24, f=40.0, sh_degree=3, n_views=1,
                 lidar_frac=0.1, dtype=np.float64):
    """Small random scene for gradient checks: Gaussians in front of 1-2 cameras."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1, 1, (n, 3)) * [1.2, 0.9, 0.8] + [0, 0, 3.0]
    ls = rng.normal(-2.3, 0.3, (n, 3))
    q = rng.normal(size=(n, 4))
    logits = rng.normal(0, 1.5, n)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0, 0.3, (n, k, 3))
    sh[:, 0, :] = rng.normal(0, 1.0, (n, 3))
    cams = [camera(f=f, width=width, height=height)]
    if n_views > 1:
        a = math.radians(12)
        R = np.array([[math.cos(a), 0, -math.sin(a)], [0, 1, 0], [math.sin(a), 0, math.cos(a)]])
        cams.append(camera(R=R, t=np.array([0.3, -0.1, 0.2]), f=f * 1.1, width=width + 8,
                           height=height - 4))
    gt = [rng.uniform(0, 1, (3, c.height, c.width)) for c in cams]
    lidar = []
    for c in cams:
        m = max(1, int(lidar_frac * c.width * c.height))
        pix = np.sort(rng.choice(c.width * c.height, m, replace=False)).astype(np.int32)
        lidar.append({"pix": pix, "depth": rng.uniform(2.5, 3.5, m), "sigma": rng.uniform(0.5, 1.0, m)})
    return scene(means, ls, q, logits, sh=sh, cams=cams, sh_degree=sh_degree, gt=gt,
                 lidar=lidar, dtype=dtype)
