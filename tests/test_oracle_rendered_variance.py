"""Pins for the rendered-variance reading of the LiDAR term (Sec. III-C: the renderer
predicts N(mu_u, sigma_u^2) per pixel; here sigma_u^2 = sum w z^2 - mu_u^2 + floor, the variance
of the rendered depth distribution): closed forms for one and two Gaussians, the Jensen
bound of the variance, and frozen-decision finite differences of every gradient."""
import math

import numpy as np

from oracle.render import frozen_objective, loss_and_grads, render
from oracle.settings import RenderSettings
from tests.oracle_helpers import camera, logit, random_scene, scene


def _kl(m1, s1, m2, s2):
    return math.log(s2 / s1) + (s1 * s1 + (m1 - m2) ** 2) / (2 * s2 * s2) - 0.5


def test_single_and_two_gaussian_closed_forms():
    cam = camera(f=100.0, width=4, height=2, cx=1.5, cy=0.5)   # pixel (1, 0) on the axis
    gt = np.zeros((3, 2, 4))
    D, sig, floor = 1.7, 0.05, 1e-4
    lid = {"pix": np.array([1], np.int32), "depth": np.array([D]), "sigma": np.array([sig])}
    s = RenderSettings(blur=0.0)
    # one Gaussian: mu = o z, D2 = o z^2, variance o (1 - o) z^2
    o, z = 0.6, 2.0
    sc = scene([[0, 0, z]], log_scales=[[-6.0] * 3], logits=[logit(o)], rgb=[[0.5, 0.5, 0.5]], cams=[cam],
               gt=[gt], lidar=[lid])
    r = loss_and_grads(sc, s, w_l1=0.0, lam=1.5, sigma_mode="rendered", sigma_floor=floor)
    v = o * (1 - o) * z * z + floor
    assert math.isclose(r["loss"], 1.5 * _kl(D, sig, o * z, math.sqrt(v)), rel_tol=1e-12)
    # two Gaussians on the axis: w1 = o1, w2 = o2 (1 - o1)
    o1, z1, o2, z2 = 0.4, 1.5, 0.7, 3.0
    sc2 = scene([[0, 0, z1], [0, 0, z2]], log_scales=[[-6.0] * 3] * 2, logits=[logit(o1), logit(o2)],
                rgb=[[0.5] * 3] * 2, cams=[cam], gt=[gt], lidar=[lid])
    r2 = loss_and_grads(sc2, s, w_l1=0.0, lam=1.0, sigma_mode="rendered", sigma_floor=floor)
    w1, w2 = o1, o2 * (1 - o1)
    mu = w1 * z1 + w2 * z2
    v2 = w1 * z1 * z1 + w2 * z2 * z2 - mu * mu + floor
    assert math.isclose(r2["loss"], _kl(D, sig, mu, math.sqrt(v2)), rel_tol=1e-12)
    # the fixed-variance reading is unchanged by the new output
    rf = loss_and_grads(sc2, s, w_l1=0.0, lam=1.0)
    assert math.isclose(rf["loss"], (D - mu) ** 2 / (2 * sig * sig), rel_tol=1e-12)


def test_rendered_variance_is_non_negative():
    """sum w z^2 >= (sum w z)^2 / sum w >= (sum w z)^2 since sum w = A <= 1 (Jensen)."""
    sc = random_scene(61, n=80, width=24, height=20)
    for v in render(sc, RenderSettings()):
        var = v["depth2"] - v["depth"] ** 2
        assert var.min() >= -1e-12
        assert np.all(v["alpha"] <= 1 + 1e-12)


def test_rendered_variance_gradients_match_frozen_decision_finite_differences():
    sc = random_scene(71, n=60, n_views=2)
    s = RenderSettings()
    kw = dict(lam=0.8, sigma_mode="rendered", sigma_floor=1e-3)
    r = loss_and_grads(sc, s, **kw)
    rng = np.random.default_rng(72)
    h = 1e-6
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        arr = getattr(sc, name)
        g = r["grads"][name]
        for flat in list(np.argsort(-np.abs(g).ravel())[:3]) + list(rng.choice(g.size, 3, replace=False)):
            old = arr.flat[flat]
            arr.flat[flat] = old + h
            lp = frozen_objective(sc, r["decisions"], s, **kw)
            arr.flat[flat] = old - h
            lm = frozen_objective(sc, r["decisions"], s, **kw)
            arr.flat[flat] = old
            fd = (lp - lm) / (2 * h)
            tol = 1e-6 * abs(g.flat[flat]) + 1e-9 * np.abs(g).max() + 50 * 2.2e-16 * max(abs(r["loss"]), 1) / h
            assert abs(fd - g.flat[flat]) <= tol, (name, flat, fd, g.flat[flat])
    for b in range(2):
        for j in range(6):
            d = np.zeros((2, 6))
            d[b, j] = h
            fd = (frozen_objective(sc, r["decisions"], s, deltas=d, **kw) -
                  frozen_objective(sc, r["decisions"], s, deltas=-d, **kw)) / (2 * h)
            g = r["pose"][b, j]
            assert abs(fd - g) <= 1e-6 * abs(g) + 1e-9 * np.abs(r["pose"]).max() + 1e-11, (b, j, fd, g)
