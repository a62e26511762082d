"""Pins for the oracle's projection (Sec. III-B, Sigma' = J W Sigma W^T J^T) and its
brute-force front-to-back compositing (standard 3DGS compositing, Sec. III-B)."""
import math

import numpy as np
import pytest
import torch

from oracle.render import (composite_decisions, composite_eval, depth_key_uncertain, leaves, project,
                           render)
from oracle.settings import RenderSettings
from paper_2510_26358_amd.scenes import tiny_scene
from tests.oracle_helpers import camera, logit, scene

DT = torch.float64


def _proj(sc, s, b=0):
    p = leaves(sc, requires_grad=False)
    return project(p, sc.cameras[b], p["pose_delta"][b], s, sc.sh_degree)


def test_on_axis_projection_closed_form():
    """R_b = I, identity rotation, no blur: Sigma' = diag(fx^2 e^{2sx}, fy^2 e^{2sy}) / z^2."""
    z = 3.7
    s = RenderSettings(blur=0.0)
    ls = np.array([[-2.0, -1.5, -3.0]])
    sc = scene([[0, 0, z]], log_scales=ls, cams=[camera(f=120.0, fy=90.0, width=64, height=48)])
    pr = _proj(sc, s)
    S2 = pr["cov2d"][0].numpy()
    expect = np.diag([120.0 ** 2 * math.exp(2 * ls[0, 0]), 90.0 ** 2 * math.exp(2 * ls[0, 1])]) / z ** 2
    assert np.allclose(S2, expect, rtol=1e-13, atol=0)
    assert np.isclose(pr["u"][0].item(), 32.0) and np.isclose(pr["v"][0].item(), 24.0)
    conic = pr["conic"][0].numpy()
    K = np.array([[conic[0], conic[1]], [conic[1], conic[2]]])
    assert np.allclose(K @ S2, np.eye(2), atol=1e-12)


def _pinhole(Xw, R, t, f, fy, cx, cy):
    Xc = Xw @ R.T + t
    return np.stack([f * Xc[:, 0] / Xc[:, 2] + cx, fy * Xc[:, 1] / Xc[:, 2] + cy], 1)


@pytest.mark.parametrize("blur", [0.0, 0.3])
def test_projected_covariance_matches_monte_carlo_of_the_pinhole(blur):
    """Sample 3D points from N(mu, Sigma), push them through the actual pinhole map of a
    rotated, translated camera and compare the empirical image covariance (plus blur) with
    the oracle's Sigma'.  Catches a wrong J, a transposed W or a dropped term."""
    rng = np.random.default_rng(5)
    a = 0.4
    R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    R = R @ np.array([[1, 0, 0], [0, math.cos(0.2), -math.sin(0.2)], [0, math.sin(0.2), math.cos(0.2)]])
    t = np.array([0.2, -0.3, 1.0])
    cam = camera(R=R, t=t, f=300.0, fy=280.0, width=400, height=300, cx=190.0, cy=160.0)
    mu = np.array([0.4, 0.2, 3.0])
    ls = np.array([-4.6, -5.3, -4.9])
    q = np.array([0.8, 0.3, -0.4, 0.2])
    sc = scene([mu], log_scales=[ls], quats=[q], cams=[cam])
    pr = _proj(sc, RenderSettings(blur=blur))
    S2 = pr["cov2d"][0].numpy()
    qn = q / np.linalg.norm(q)
    w, x, y, z = qn
    Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    L = Rq @ np.diag(np.exp(ls))
    X = mu + rng.normal(size=(2_000_000, 3)) @ L.T
    uv = _pinhole(X, R, t, 300.0, 280.0, 190.0, 160.0)
    emp = np.cov(uv.T) + blur * np.eye(2)
    assert np.allclose(S2, emp, rtol=5e-3, atol=2e-3 * np.abs(S2).max())
    uv0 = _pinhole(mu[None], R, t, 300.0, 280.0, 190.0, 160.0)[0]
    assert np.allclose([pr["u"][0].item(), pr["v"][0].item()], uv0, atol=1e-12)


def test_jacobian_matches_finite_differences_of_the_pinhole():
    rng = np.random.default_rng(6)
    for _ in range(5):
        xc = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(2, 5)])
        f, fy = 200.0, 180.0
        h = 1e-6
        Jfd = np.zeros((2, 3))
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            Jfd[:, j] = (_pinhole((xc + e)[None], np.eye(3), np.zeros(3), f, fy, 0, 0)[0] -
                         _pinhole((xc - e)[None], np.eye(3), np.zeros(3), f, fy, 0, 0)[0]) / (2 * h)
        # the oracle's Sigma' for an isotropic tiny Gaussian equals s^2 J J^T (blur 0)
        sc = scene([xc], log_scales=[[-3.0] * 3], cams=[camera(f=f, fy=fy, width=2000, height=2000)])
        S2 = _proj(sc, RenderSettings(blur=0.0))["cov2d"][0].numpy()
        assert np.allclose(S2, math.exp(-6.0) * Jfd @ Jfd.T, rtol=1e-7)


def test_view_direction_enters_the_colour_through_sh():
    """Degree-1 SH with only the m = +1 coefficient (-x lobe) set: a Gaussian straight
    ahead of a camera looking along +x world gets rgb = 0.5 + f * Y_11((1,0,0))."""
    c1 = math.sqrt(3 / (4 * math.pi))
    # camera at (1, 2, 0) looking along world +x: rows (right, down, forward)
    R = np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])
    C = np.array([1.0, 2.0, 0.0])
    cam = camera(R=R, t=-R @ C, f=50.0, width=40, height=40)
    sh = np.zeros((1, 4, 3))
    sh[0, 3, :] = [-0.2, 0.1, 0.3]
    sc = scene([C + [4.0, 0.0, 0.0]], sh=sh, sh_degree=1, cams=[cam])
    rgb = _proj(sc, RenderSettings())["rgb"][0].numpy()
    assert np.allclose(rgb, np.maximum(0.0, 0.5 + sh[0, 3] * (-c1)), atol=1e-14)


def test_culling_near_plane_and_faint_gaussians():
    s = RenderSettings()
    sc = scene([[0, 0, 0.1], [0, 0, 0.25], [0, 0, 2.0], [0, 0, 2.0]],
               logits=[3.0, 3.0, logit(0.5 / 255), logit(2.0 / 255)])
    valid = _proj(sc, s)["valid"].numpy()
    assert valid.tolist() == [False, True, False, True]


# ---------------------------------------------------------------- compositing
def _render_pixels(sc, px, py, s=None):
    s = s or RenderSettings()
    cam = sc.cameras[0]
    pix = np.asarray(py) * cam.width + np.asarray(px)
    return render(sc, s, pixels=[pix])[0]


def test_single_gaussian_at_pixel_centre():
    """alpha = o, C = o rgb, A = o, D = o z for a Gaussian centred on a pixel centre."""
    o = 0.7
    rgb = [0.2, 0.6, 0.9]
    cam = camera(width=32, height=24, cx=16.5, cy=12.5)  # (u, v) = (16.5, 12.5): pixel (16, 12)
    sc = scene([[0, 0, 2.5]], logits=[logit(o)], rgb=[rgb], cams=[cam])
    r = _render_pixels(sc, [16], [12])
    assert np.allclose(r["alpha"], o, atol=1e-15)
    assert np.allclose(r["rgb"][0], o * np.array(rgb), atol=1e-14)
    assert np.allclose(r["depth"], o * 2.5, atol=1e-14)
    assert np.allclose(r["T"], 1 - o, atol=1e-15)


def test_alpha_is_clamped_at_alpha_max():
    cam = camera(width=32, height=24, cx=16.5, cy=12.5)
    sc = scene([[0, 0, 2.0]], logits=[logit(0.999)], rgb=[[1, 1, 1]], cams=[cam])
    r = _render_pixels(sc, [16], [12])
    assert np.allclose(r["alpha"], 0.99, atol=1e-15)


def test_two_gaussians_over_operator_in_depth_order():
    """The nearer Gaussian is composited first, whatever the array order:
    C = a1 c1 + (1 - a1) a2 c2 with 1 the nearer one."""
    cam = camera(width=32, height=24, cx=16.5, cy=12.5)
    o_far, o_near = 0.5, 0.4
    c_far, c_near = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    sc = scene([[0, 0, 4.0], [0, 0, 2.0]], logits=[logit(o_far), logit(o_near)],
               rgb=[c_far, c_near], cams=[cam])
    r = _render_pixels(sc, [16], [12])
    expect = o_near * c_near + (1 - o_near) * o_far * c_far
    assert np.allclose(r["rgb"][0], expect, atol=1e-14)
    assert np.allclose(r["depth"], o_near * 2.0 + (1 - o_near) * o_far * 4.0, atol=1e-14)
    assert np.allclose(r["alpha"], o_near + (1 - o_near) * o_far, atol=1e-15)


def test_equal_depths_composite_in_index_order_and_are_not_ambiguous():
    """Two Gaussians at exactly the same depth are ordered by index (the depth key is the
    float32 depth, ties broken by the Gaussian index), whatever their colours: swapping the
    array order swaps which one is in front.  Every float64 evaluation of an exactly
    representable depth rounds to the same key, so the pixel is not ambiguous."""
    cam = camera(width=32, height=24, cx=16.5, cy=12.5)
    red, blue = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    for first, second in [(red, blue), (blue, red)]:
        sc = scene([[0, 0, 3.0], [0, 0, 3.0]], logits=[logit(0.5), logit(0.4)], rgb=[first, second],
                   cams=[cam], dtype=np.float32)
        r = _render_pixels(sc, [16], [12])
        assert not r["ambiguous"][0]
        assert np.allclose(r["rgb"][0], 0.5 * first + 0.5 * 0.4 * second, atol=1e-7)


def test_depth_on_a_float32_rounding_boundary_is_ambiguous():
    """mu_z = 1 + 2^-23 (a float32) seen from t_z = 2 has depth 3 + 2^-23, the midpoint of
    the float32 values 3 and 3 + 2^-22: its key depends on the last bit of the evaluation.
    Next to a Gaussian at depth exactly 3 the order of the two can change, so the pixel is
    flagged; next to one at 2.5 it cannot, and a depth one float32 step away is certain."""
    z_mid = 3.0 + 2.0 ** -23
    assert depth_key_uncertain([z_mid], [1e-15])[0]
    assert not depth_key_uncertain([3.0], [1e-15])[0]
    assert not depth_key_uncertain([3.0 + 2.0 ** -22], [1e-15])[0]
    assert not depth_key_uncertain([z_mid + 1e-12], [1e-15])[0]
    cam = camera(t=[0.0, 0.0, 2.0], width=32, height=24, cx=16.5, cy=12.5, dtype=np.float32)

    def pixel(mu_first, mu_second):
        sc = scene([[0, 0, mu_first], [0, 0, mu_second]], logits=[logit(0.5), logit(0.4)], cams=[cam],
                   dtype=np.float32)
        assert sc.means[0, 2] == np.float32(mu_first)
        r = _render_pixels(sc, [16], [12])
        assert r["count"][0] == 2
        return bool(r["ambiguous"][0])

    assert pixel(1.0 + 2.0 ** -23, 1.0)
    assert not pixel(1.0 + 2.0 ** -23, 0.5)
    assert not pixel(1.0 + 2.0 ** -22, 1.0)


def test_transmittance_stop_excludes_the_crossing_gaussian():
    """Five stacked Gaussians with alpha = 0.95: T goes 1, .05, .0025, 1.25e-4, then the
    fourth would give 6.25e-6 < 1e-4, so it and the rest are excluded: 3 contributors."""
    cam = camera(width=32, height=24, cx=16.5, cy=12.5)
    zs = [2.0, 2.5, 3.0, 3.5, 4.0]
    sc = scene([[0, 0, z] for z in zs], logits=[logit(0.95)] * 5,
               rgb=[[1, 1, 1]] * 5, cams=[cam])
    r = _render_pixels(sc, [16], [12])
    assert r["count"][0] == 3
    assert np.isclose(r["T"][0], 0.05 ** 3, rtol=1e-13)
    assert np.isclose(r["alpha"][0], 1 - 0.05 ** 3, rtol=1e-13)
    w = [0.95, 0.95 * 0.05, 0.95 * 0.05 ** 2]
    assert np.isclose(r["depth"][0], sum(wi * z for wi, z in zip(w, zs)), rtol=1e-13)


def test_faint_gaussian_below_alpha_min_is_skipped():
    cam = camera(width=32, height=24, cx=16.5, cy=12.5)
    # off-centre so that o * exp(power) < 1/255 at the pixel while o > 1/255
    sc = scene([[0.0, 0, 2.0]], log_scales=[[-4.0] * 3], logits=[logit(0.05)], rgb=[[1, 1, 1]],
               cams=[camera(width=32, height=24, cx=20.5, cy=12.5)])
    r = _render_pixels(sc, [16], [12])
    assert r["count"][0] == 0 and r["alpha"][0] == 0.0 and r["T"][0] == 1.0


def _naive_pixel(sc, b, px, py, s):
    """Scalar double loop straight from the definition, for a handful of pixels."""
    pr = _proj(sc, s, b)
    u, v = pr["u"].numpy(), pr["v"].numpy()
    con, o, rgb, z = pr["conic"].numpy(), pr["o"].numpy(), pr["rgb"].numpy(), pr["z"].numpy()
    valid = pr["valid"].numpy()
    cand = []
    for i in range(len(u)):
        if not valid[i]:
            continue
        dx, dy = u[i] - (px + 0.5), v[i] - (py + 0.5)
        pw = -0.5 * (con[i, 0] * dx * dx + con[i, 2] * dy * dy) - con[i, 1] * dx * dy
        if pw > 0:
            continue
        al = min(s.alpha_max, o[i] * math.exp(pw))
        if al >= s.alpha_min:
            cand.append((np.float32(z[i]), i, al))
    cand.sort(key=lambda e: (e[0], e[1]))
    T, C, D, A = 1.0, np.zeros(3), 0.0, 0.0
    for _, i, al in cand:
        Tn = T * (1 - al)
        if Tn < s.t_min:
            break
        w = al * T
        C += w * rgb[i]
        D += w * z[i]
        A += w
        T = Tn
    return C + T * np.array(s.bg), D, A, T


def test_vectorised_oracle_equals_scalar_loop_on_the_tiny_scene():
    sc = tiny_scene()
    s = RenderSettings(bg=(0.1, 0.2, 0.3))
    rng = np.random.default_rng(7)
    px = rng.integers(0, 128, 40)
    py = rng.integers(0, 96, 40)
    r = _render_pixels(sc, px, py, s)
    for k in range(len(px)):
        C, D, A, T = _naive_pixel(sc, 0, px[k], py[k], s)
        assert np.allclose(r["rgb"][k], C, atol=1e-13)
        assert np.isclose(r["depth"][k], D, atol=1e-12)
        assert np.isclose(r["alpha"][k], A, atol=1e-14)
        assert np.isclose(r["T"][k], T, atol=1e-14)


def test_accumulated_alpha_plus_final_transmittance_is_one():
    sc = tiny_scene()
    r = render(sc, RenderSettings())[0]
    assert np.abs(r["alpha"] + r["T"] - 1.0).max() <= 1e-12
    assert (r["T"] >= 1e-4).all()


def test_gaussian_array_order_does_not_change_the_image():
    sc = tiny_scene()
    rng = np.random.default_rng(8)
    perm = rng.permutation(sc.n)
    sc2 = sc.copy()
    sc2.means, sc2.log_scales, sc2.quats = sc.means[perm], sc.log_scales[perm], sc.quats[perm]
    sc2.opacity_logits, sc2.sh = sc.opacity_logits[perm], sc.sh[perm]
    pix = rng.choice(128 * 96, 300, replace=False)
    a = render(sc, pixels=[pix])[0]
    b = render(sc2, pixels=[pix])[0]
    ok = ~(a["ambiguous"] | b["ambiguous"])
    assert np.allclose(a["rgb"][ok], b["rgb"][ok], atol=1e-13)
    assert np.allclose(a["depth"][ok], b["depth"][ok], atol=1e-12)


def test_background_enters_through_final_transmittance():
    sc = tiny_scene()
    pix = np.arange(0, 128 * 96, 97)
    a = render(sc, RenderSettings(), pixels=[pix])[0]
    bg = (0.3, 0.5, 0.7)
    b = render(sc, RenderSettings(bg=bg), pixels=[pix])[0]
    assert np.allclose(b["rgb"] - a["rgb"], a["T"][:, None] * np.array(bg), atol=1e-14)
