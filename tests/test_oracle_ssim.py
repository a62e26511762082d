"""Pins for the oracle's SSIM (D-SSIM part of L_3DGS, Sec. III-C) and for the loss that
uses it: a library special case (the Gaussian blur), brute-force windowed statistics,
invariants, a closed form, and finite differences of the whole loss."""
import math

import numpy as np
import scipy.ndimage
import torch

from oracle.render import frozen_objective, loss_and_grads
from oracle.settings import RenderSettings
from oracle.ssim import C1, C2, blur, gaussian_window, ssim_map
from tests.oracle_helpers import random_scene

DT = torch.float64


def test_blur_is_the_zero_padded_gaussian_filter():
    """Library special case: scipy's Gaussian filter with zero ('constant') padding, the same
    sigma and a window truncated at radius 5 (truncate * sigma + 0.5 -> 5)."""
    rng = np.random.default_rng(0)
    img = rng.random((3, 23, 31))
    ref = np.stack([scipy.ndimage.gaussian_filter(c, sigma=1.5, mode="constant", cval=0.0,
                                                  truncate=5.0 / 1.5) for c in img])
    got = blur(torch.tensor(img)).numpy()
    assert np.allclose(got, ref, rtol=0, atol=1e-14)
    w = gaussian_window()
    assert len(w) == 11 and math.isclose(float(w.sum()), 1.0, rel_tol=1e-15)
    assert torch.allclose(w, w.flip(0), rtol=0, atol=0)


def _brute_stats(x, y, py, px, r=5, sigma=1.5):
    """Weighted local statistics at one pixel straight from the 2D window (zero outside)."""
    num = 0.0
    mx = my = exx = eyy = exy = 0.0
    ws = 0.0
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            ws += math.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            w = math.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma)) / ws
            yy, xx = py + dy, px + dx
            if 0 <= yy < x.shape[0] and 0 <= xx < x.shape[1]:
                a, b = x[yy, xx], y[yy, xx]
            else:
                a = b = 0.0
            mx += w * a
            my += w * b
            exx += w * a * a
            eyy += w * b * b
            exy += w * a * b
            num += 1
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def test_ssim_map_matches_brute_force_windows():
    rng = np.random.default_rng(1)
    x = rng.random((2, 17, 13))
    y = np.clip(x + 0.2 * rng.standard_normal(x.shape), 0, 1)
    s = ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    for (c, py, px) in [(0, 0, 0), (0, 8, 6), (1, 16, 12), (1, 3, 10), (0, 12, 1)]:
        assert math.isclose(s[c, py, px], _brute_stats(x[c], y[c], py, px), rel_tol=1e-12, abs_tol=1e-13)


def test_ssim_invariants_and_constant_closed_form():
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.random((3, 20, 24)))
    y = torch.tensor(rng.random((3, 20, 24)))
    assert torch.allclose(ssim_map(x, x), torch.ones_like(x), rtol=0, atol=1e-12)
    assert torch.allclose(ssim_map(x, y), ssim_map(y, x), rtol=0, atol=1e-14)
    s = ssim_map(x, y)
    assert float(s.max()) <= 1.0 + 1e-12
    # constant images: away from the zero padding the variances vanish, so
    # s = (2ab + C1) / (a^2 + b^2 + C1)
    a, b = 0.3, 0.7
    xc = torch.full((1, 21, 21), a, dtype=DT)
    yc = torch.full((1, 21, 21), b, dtype=DT)
    sc = ssim_map(xc, yc)[0, 5:16, 5:16]
    assert torch.allclose(sc, torch.full_like(sc, (2 * a * b + C1) / (a * a + b * b + C1)), rtol=1e-12, atol=0)


def test_loss_with_ssim_reduces_to_l1_and_matches_finite_differences():
    sc = random_scene(31, n=120, sh_degree=1, n_views=1, width=40, height=28, f=36.0)
    s = RenderSettings()
    r0 = loss_and_grads(sc, s, lam=0.0)
    r00 = loss_and_grads(sc, s, lam=0.0, ssim_w=0.0)
    assert r0["loss"] == r00["loss"]
    lam_s = 0.2
    r = loss_and_grads(sc, s, lam=0.5, ssim_w=lam_s)
    # value: (1 - l) L1 + l (1 - mean ssim) + lidar, assembled from a separate evaluation
    out = r["views"][0]
    img = np.zeros((3, sc.cameras[0].height * sc.cameras[0].width))
    img[:, out["pix"]] = out["rgb"].T
    cam = sc.cameras[0]
    smap = ssim_map(torch.tensor(img.reshape(3, cam.height, cam.width)), torch.tensor(sc.gt_rgb[0])).numpy()
    l1 = np.abs(img - sc.gt_rgb[0].reshape(3, -1)).mean()
    r_l1_lidar = loss_and_grads(sc, s, lam=0.5, w_l1=0.0)["loss"]
    expect = (1 - lam_s) * l1 + lam_s * (1 - smap.mean()) + r_l1_lidar
    assert math.isclose(r["loss"], expect, rel_tol=1e-12)
    # gradients: frozen-decision central differences on a few coordinates
    rng = np.random.default_rng(5)
    h = 1e-6
    for name in ("means", "sh", "opacity_logits"):
        arr = getattr(sc, name)
        g = r["grads"][name]
        for flat in list(np.argsort(-np.abs(g).ravel())[:2]) + list(rng.choice(g.size, 2, replace=False)):
            old = arr.flat[flat]
            arr.flat[flat] = old + h
            fp = frozen_objective(sc, r["decisions"], s, lam=0.5, ssim_w=lam_s)
            arr.flat[flat] = old - h
            fm = frozen_objective(sc, r["decisions"], s, lam=0.5, ssim_w=lam_s)
            arr.flat[flat] = old
            fd = (fp - fm) / (2 * h)
            tol = 1e-6 * max(1.0, abs(fd)) + 50 * 2.2e-16 * abs(r["loss"]) / h
            assert abs(g.flat[flat] - fd) <= tol, (name, flat, g.flat[flat], fd)
