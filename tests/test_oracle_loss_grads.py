"""Pins for the oracle's loss (Sec. III-C: L1 part of L_3DGS plus the LiDAR KL term) and
for its float64 gradients to Gaussians and to SE(3) camera poses (poses refined by
back-propagation through the projection, Sec. III-C and abstract)."""
import math

import numpy as np
import pytest
import scipy.integrate
import torch

from oracle.geometry import quat_to_rotmat
from oracle.render import frozen_objective, kl_normal, loss_and_grads, render
from oracle.settings import RenderSettings
from tests.oracle_helpers import camera, logit, random_scene, scene

DT = torch.float64


def _kl(m1, s1, m2, s2):
    return float(kl_normal(torch.tensor(m1, dtype=DT), torch.tensor(s1, dtype=DT),
                           torch.tensor(m2, dtype=DT), torch.tensor(s2, dtype=DT)))


def test_kl_closed_forms_and_numerical_integral():
    assert _kl(3.0, 0.2, 3.0, 0.2) == 0.0
    assert math.isclose(_kl(3.0, 0.2, 3.5, 0.2), 0.5 ** 2 / (2 * 0.04), rel_tol=1e-14)
    for (m1, s1, m2, s2) in [(0.0, 1.0, 1.0, 2.0), (5.0, 0.3, 4.2, 0.7), (1.0, 2.0, 0.0, 0.5)]:
        p = lambda x: math.exp(-(x - m1) ** 2 / (2 * s1 * s1)) / (s1 * math.sqrt(2 * math.pi))
        lq = lambda x: -(x - m2) ** 2 / (2 * s2 * s2) - math.log(s2 * math.sqrt(2 * math.pi))
        lp = lambda x: -(x - m1) ** 2 / (2 * s1 * s1) - math.log(s1 * math.sqrt(2 * math.pi))
        val, _ = scipy.integrate.quad(lambda x: p(x) * (lp(x) - lq(x)), m1 - 30 * s1, m1 + 30 * s1,
                                      limit=400, epsabs=1e-13)
        assert math.isclose(_kl(m1, s1, m2, s2), val, rel_tol=1e-9, abs_tol=1e-12)


def test_loss_closed_form_single_gaussian():
    """One Gaussian on a pixel centre of a 4x2 image: per-pixel values are known in closed
    form at that pixel, background 0 elsewhere is checked through the L1 mean."""
    o, z = 0.6, 2.0
    rgb = np.array([0.2, 0.5, 0.8])
    cam = camera(f=100.0, width=4, height=2, cx=1.5, cy=0.5)   # centred on pixel (1, 0)
    gt = np.full((3, 2, 4), 0.25)
    lid = {"pix": np.array([1], np.int32), "depth": np.array([1.5]), "sigma": np.array([0.1])}
    sc = scene([[0, 0, z]], log_scales=[[-6.0] * 3], logits=[logit(o)], rgb=[rgb], cams=[cam],
               gt=[gt], lidar=[lid])
    r = loss_and_grads(sc, RenderSettings(blur=0.0), w_l1=0.8, lam=2.0)
    # only pixel (1, 0) is covered (tiny Gaussian): C = o rgb there, 0 elsewhere
    l1 = (np.abs(o * rgb - 0.25).sum() + 7 * 3 * 0.25) * 0.8 / (3 * 8)
    lid_term = 2.0 * (1.5 - o * z) ** 2 / (2 * 0.1 ** 2)
    assert math.isclose(r["loss"], l1 + lid_term, rel_tol=1e-12)


def _fd_check(sc, s, names, rng, n_checks=8, h=1e-6, lam=1.0, masks=None, upstream=None):
    r = loss_and_grads(sc, s, masks=masks, lam=lam, upstream=upstream)
    dec = r["decisions"]
    for name in names:
        arr = getattr(sc, name)
        g = r["grads"][name]
        flat = np.argsort(-np.abs(g).ravel())[: n_checks // 2]
        flat = np.concatenate([flat, rng.choice(g.size, n_checks - len(flat), replace=False)])
        for f in flat:
            idx = np.unravel_index(f, arr.shape)
            old = arr[idx]
            arr[idx] = old + h
            lp = frozen_objective(sc, dec, s, masks=masks, lam=lam, upstream=upstream)
            arr[idx] = old - h
            lm = frozen_objective(sc, dec, s, masks=masks, lam=lam, upstream=upstream)
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            scale = max(np.abs(g).max() * 1e-3, 1e-9)
            roundoff = 50 * np.finfo(np.float64).eps * max(abs(r["loss"]), 1.0) / h
            assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx]) + 1e-6 * scale + roundoff, (name, idx, fd, g[idx])
    return r


@pytest.mark.parametrize("n_views", [1, 2])
def test_gaussian_gradients_match_frozen_decision_finite_differences(n_views):
    sc = random_scene(11 + n_views, n_views=n_views)
    rng = np.random.default_rng(12)
    _fd_check(sc, RenderSettings(bg=(0.2, 0.1, 0.4)),
              ["means", "log_scales", "quats", "opacity_logits", "sh"], rng, lam=0.7)


def test_pose_gradients_match_frozen_decision_finite_differences():
    sc = random_scene(21, n_views=2)
    s = RenderSettings()
    r = loss_and_grads(sc, s, lam=0.5)
    h = 1e-6
    for b in range(2):
        for j in range(6):
            d = np.zeros((2, 6))
            d[b, j] = h
            lp = frozen_objective(sc, r["decisions"], s, lam=0.5, deltas=d)
            lm = frozen_objective(sc, r["decisions"], s, lam=0.5, deltas=-d)
            fd = (lp - lm) / (2 * h)
            g = r["pose"][b, j]
            assert abs(fd - g) <= 1e-6 * abs(g) + 1e-9 * np.abs(r["pose"]).max() + 1e-12, (b, j, fd, g)


def test_frozen_objective_keeps_the_l1_signs_of_the_forward_pass():
    """A target a hair away from the rendered colour (1e-9 beyond it, well inside what a pose
    step of 1e-6 moves it) puts a kink of |C - C_gt| inside the finite-difference interval:
    with the signs of the forward pass kept, the difference quotient equals the gradient
    sign(C - C_gt) dC/d delta; evaluated with fresh signs it would not."""
    sc = random_scene(23, n_views=1)
    s = RenderSettings()
    r0 = render(sc, s)[0]
    cam = sc.cameras[0]
    gt = np.asarray(sc.gt_rgb[0], np.float64).copy()
    # the pixel with the largest colour: its red channel's target sits 1e-9 above the render
    p = int(np.argmax(r0["rgb"][:, 0]))
    gt.reshape(3, -1)[0, p] = r0["rgb"][p, 0] + 1e-9
    r = loss_and_grads(sc, s, gt=[gt], lam=0.0)
    assert r["decisions"][0].l1_sign is not None
    h = 1e-6
    for j in range(6):
        d = np.zeros((1, 6))
        d[0, j] = h
        lp = frozen_objective(sc, r["decisions"], s, gt=[gt], lam=0.0, deltas=d)
        lm = frozen_objective(sc, r["decisions"], s, gt=[gt], lam=0.0, deltas=-d)
        fd = (lp - lm) / (2 * h)
        g = r["pose"][0, j]
        assert abs(fd - g) <= 1e-6 * abs(g) + 1e-9 * np.abs(r["pose"]).max() + 1e-12, (j, fd, g)
    # the kink is real: with the signs recomputed at +-h the quotient moves off the gradient
    off = 0.0
    for j in range(6):
        d = np.zeros((1, 6))
        d[0, j] = h
        lp = loss_and_grads(sc, s, gt=[gt], lam=0.0, deltas=d)["loss"]
        lm = loss_and_grads(sc, s, gt=[gt], lam=0.0, deltas=-d)["loss"]
        off = max(off, abs((lp - lm) / (2 * h) - r["pose"][0, j]))
    assert off > 1e-6 * np.abs(r["pose"]).max()


def test_upstream_mode_gradients_match_finite_differences():
    sc = random_scene(31, n=40)
    rng = np.random.default_rng(32)
    cam = sc.cameras[0]
    up = [{"rgb": rng.normal(size=(3, cam.height, cam.width)),
           "depth": rng.normal(size=(cam.height, cam.width)),
           "alpha": rng.normal(size=(cam.height, cam.width))}]
    _fd_check(sc, RenderSettings(), ["means", "opacity_logits", "sh"], rng, upstream=up)


def test_pose_translation_gradient_equals_rotated_sum_of_mean_gradients():
    """Moving the camera by rho is the same as moving every mean by -R^T rho, so
    dL/drho = R_b sum_i dL/dmu_i (one view)."""
    sc = random_scene(41, n_views=1)
    r = loss_and_grads(sc, RenderSettings(), lam=1.0)
    R = sc.cameras[0].R.astype(np.float64)
    assert np.allclose(r["pose"][0, :3], R @ r["grads"]["means"].sum(0), rtol=1e-10, atol=1e-14)


def test_quaternion_gradient_is_orthogonal_to_the_quaternion():
    sc = random_scene(51)
    r = loss_and_grads(sc, RenderSettings())
    gq = r["grads"]["quats"]
    dots = (gq * sc.quats).sum(1)
    assert np.abs(dots).max() <= 1e-12 * max(np.abs(gq).max(), 1e-30) * 10


def test_dc_colour_gradient_equals_visibility_weights():
    """With objective sum_p C_r(p) and unclamped colours, dL/df_dc,r(i) = Y_00 sum_p w_i(p).
    The weights are measured independently by re-rendering with Gaussian i alone carrying
    colour 1 in channel r (linearity of C in the colours)."""
    sc = random_scene(61, n=25, sh_degree=0)
    sc.sh[:, 0, :] = (0.5 - 0.5) / 0.28209479177387814 + 0.1  # keep colours unclamped (~0.53)
    cam = sc.cameras[0]
    up = [{"rgb": np.stack([np.ones((cam.height, cam.width)), np.zeros((cam.height, cam.width)),
                            np.zeros((cam.height, cam.width))]),
           "depth": np.zeros((cam.height, cam.width)), "alpha": np.zeros((cam.height, cam.width))}]
    r = loss_and_grads(sc, RenderSettings(), upstream=up)
    y00 = 0.5 / math.sqrt(math.pi)
    for i in [0, 3, 7, 11, 19]:
        sc1 = sc.copy()
        sc1.sh = np.zeros_like(sc.sh)
        sc1.sh[:, 0, :] = -0.5 / y00           # every Gaussian black...
        sc1.sh[i, 0, 0] = 0.5 / y00            # ...except i, red = 1
        img = render(sc1, RenderSettings())[0]
        assert math.isclose(r["grads"]["sh"][i, 0, 0], y00 * img["rgb"][:, 0].sum(), rel_tol=1e-10,
                            abs_tol=1e-14)
