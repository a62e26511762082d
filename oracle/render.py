"""Brute-force float64 projection, compositing, loss and gradients (oracle; tests only).

Definitions (AgriGS-SLAM, Sec. III-B and III-C; constants from `RenderSettings`):

Projection of Gaussian i into view b (Sec. III-B):
    x_c = R_b mu + t_b, z = x_c.z; culled if z < z_near
    Sigma = R(q) diag(e^{2s}) R(q)^T
    J = [[fx/z, 0, -fx tx/z^2], [0, fy/z, -fy ty/z^2]], tx = z clamp(x/z, +-1.3 W/(2 fx)), ty alike
    Sigma' = J R_b Sigma R_b^T J^T + blur I   (top-left 2x2 block of J W Sigma W^T J^T)
    conic = Sigma'^{-1}; culled if det Sigma' <= 0
    (u, v) = (fx x/z + cx, fy y/z + cy)
    o = sigmoid(omega); culled if o < alpha_min
    rgb = max(0, sum_k Y_k(d) f_k + 1/2), d = unit vector from the camera centre to mu

Compositing at pixel (px, py), centre (px + 0.5, py + 0.5), over *all* surviving Gaussians:
    power = -1/2 (a dx^2 + c dy^2) - b dx dy with (dx, dy) = (u, v) - centre
    alpha = min(alpha_max, o e^power); kept if power <= 0 and alpha >= alpha_min
    kept Gaussians ordered by (float32(z), i); T = 1; for each: T' = T (1 - alpha);
    if T' < t_min stop (this one excluded); w = alpha T; C += w rgb; D += w z; A += w; T = T'
    outputs C + T bg, D (expected depth, unnormalised), A, T_final, and D2 = sum w z^2.

Loss (Sec. III-C), summed over views b:
    w_l1 [(1 - lambda_s) / (3 n_b) sum_{p in mask} sum_ch |C - C_gt|
          + lambda_s / (3 n_b) sum_{p in mask} sum_ch (1 - ssim_ch(p))]
  + lambda_L / |Omega_b| sum_{u in Omega_b} KL(N(D_L(u), sigma_L^2) || N(mu_u, sigma_u^2)),
    mu_u = D(u), sigma_u = sigma_L (fixed-variance reading) or, in the rendered-variance
    reading, sigma_u^2 = D2(u) - mu_u^2 + floor with D2 = sum w z^2 composited like the
    depth (the variance of the rendered depth distribution); lambda_s weighs the D-SSIM
    part of L_3DGS (0: L1 only), ssim the map of `oracle.ssim` over the whole rendered
    image (zero-padded windows), averaged over the mask.

Gradients: torch float64 autograd through projection and compositing with every discrete
decision (kept sets, order, stop index, alpha clamp) frozen from the forward pass; the pose
gradient is with respect to a left perturbation W_b <- Exp(delta_b) W_b, delta = (rho, phi).
The L1 term's gradient is sign(C - C_gt) dC; an objective evaluated with frozen decisions
also keeps each pixel channel's sign of C - C_gt from the forward pass, so that finite
differences of it stay on the branch the gradient is taken on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from .geometry import covariance_3d, se3_exp_torch
from .settings import RenderSettings
from .sh import real_sh
from .ssim import ssim_map, window_radius

DT = torch.float64


def kl_normal(m1, s1, m2, s2):
    """KL( N(m1, s1^2) || N(m2, s2^2) ) for univariate normals (elementwise)."""
    return torch.log(s2 / s1) + (s1 * s1 + (m1 - m2) ** 2) / (2 * s2 * s2) - 0.5


def leaves(scene, requires_grad=True, deltas=None):
    """float64 copies of the scene's parameters, as autograd leaves.  `deltas` (B, 6) are
    the pose perturbations at which to evaluate (default 0)."""
    p = {
        "means": torch.tensor(scene.means, dtype=DT),
        "log_scales": torch.tensor(scene.log_scales, dtype=DT),
        "quats": torch.tensor(scene.quats, dtype=DT),
        "opacity_logits": torch.tensor(scene.opacity_logits, dtype=DT),
        "sh": torch.tensor(scene.sh, dtype=DT),
        "pose_delta": (torch.zeros(len(scene.cameras), 6, dtype=DT) if deltas is None
                       else torch.tensor(np.asarray(deltas, np.float64))),
    }
    for v in p.values():
        v.requires_grad_(requires_grad)
    return p


def camera_pose(cam, delta):
    """World->camera (R, t) after the left perturbation Exp(delta) (float64, differentiable)."""
    R0 = torch.tensor(cam.R, dtype=DT)
    t0 = torch.tensor(cam.t, dtype=DT)
    Rd, td = se3_exp_torch(delta)
    return Rd @ R0, Rd @ t0 + td


def project(p, cam, delta, s: RenderSettings, sh_degree: int):
    """Project Gaussians [g_begin, g_end) of the parameters into camera `cam`.

    Returns a dict of per-Gaussian tensors (differentiable where continuous) and the bool
    mask `valid` (culling decisions)."""
    g0, g1 = cam.g_begin, cam.g_end
    mu = p["means"][g0:g1]
    R, t = camera_pose(cam, delta)
    xc = mu @ R.T + t
    z = xc[:, 2]
    valid = (z >= s.z_near).detach()
    zs = torch.where(valid, z, torch.ones_like(z))  # keep culled entries finite
    x, y = xc[:, 0], xc[:, 1]
    limx = s.fov_clamp * cam.width / (2.0 * cam.fx)
    limy = s.fov_clamp * cam.height / (2.0 * cam.fy)
    tx = torch.clamp(x / zs, -limx, limx) * zs
    ty = torch.clamp(y / zs, -limy, limy) * zs
    zero = torch.zeros_like(zs)
    J = torch.stack([torch.stack([cam.fx / zs, zero, -cam.fx * tx / (zs * zs)], -1),
                     torch.stack([zero, cam.fy / zs, -cam.fy * ty / (zs * zs)], -1)], -2)
    Sigma = covariance_3d(p["log_scales"][g0:g1], p["quats"][g0:g1])
    Sigma_c = R @ Sigma @ R.T
    S2 = J @ Sigma_c @ J.transpose(-1, -2)
    S2 = S2 + s.blur * torch.eye(2, dtype=DT)
    a, b, c = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    det = a * c - b * b
    valid = valid & (det > 0).detach()
    dets = torch.where(valid, det, torch.ones_like(det))
    conic = torch.stack([c / dets, -b / dets, a / dets], -1)
    u = cam.fx * x / zs + cam.cx
    v = cam.fy * y / zs + cam.cy
    o = torch.sigmoid(p["opacity_logits"][g0:g1])
    valid = valid & (o >= s.alpha_min).detach()
    # bound on the rounding error of z = R_2 . mu + t_2 in any float64 evaluation order
    # (each product exact, a few roundings of at most 2^-53 of the running sum): 2^-44 times
    # the sum of the terms' magnitudes leaves a wide margin
    with torch.no_grad():
        z_err = 2.0 ** -44 * (mu.abs() @ R[2].abs() + t[2].abs())
    centre = -(R.T @ t)
    dvec = mu - centre
    d = dvec / torch.linalg.norm(dvec, dim=-1, keepdim=True)
    Y = real_sh(sh_degree, d)                       # (n, K)
    raw = torch.einsum("nk,nkc->nc", Y, p["sh"][g0:g1]) + 0.5
    rgb = torch.clamp(raw, min=0.0)
    # footprint bounding half-extents (for the binning reference and diagnostics): the box of
    # the alpha = alpha_min level, o exp(-q/2) = alpha_min at q = 2 ln(o / alpha_min)
    with torch.no_grad():
        lnterm = torch.where(valid, 2.0 * torch.log(o.clamp_min(1e-30) / s.alpha_min), zero)
        ext = torch.stack([torch.sqrt(lnterm.clamp_min(0) * a), torch.sqrt(lnterm.clamp_min(0) * c)], -1)
    return {"u": u, "v": v, "conic": conic, "o": o, "rgb": rgb, "z": z, "valid": valid,
            "cov2d": S2, "ext": ext, "g0": g0, "z_err": z_err}


@dataclass
class Decisions:
    """Frozen per-pixel compositing decisions for a set of pixels of one view."""
    idx: np.ndarray        # (P, Kmax) int64 local Gaussian indices in composite order, -1 pad
    clamped: np.ndarray    # (P, Kmax) bool: alpha took the alpha_max clamp
    count: np.ndarray      # (P,) number of contributors
    ambiguous: np.ndarray  # (P,) bool: a decision lies within the FP32-vs-FP64 margin
    touched: list          # per pixel: local indices processed (contributors + stopper)
    l1_sign: np.ndarray = None  # (P_l1, 3) sign of C - C_gt on the L1 pixels, set by the loss


def depth_key_range(z64, z_err):
    """The float32 depth keys another float64 evaluation of z (error at most `z_err`) could
    round to: (lo, hi), equal to float32(z) unless z lies within z_err of a rounding
    boundary (the midpoint between adjacent float32 values), where the two float32 values
    beside that boundary are both possible."""
    z64 = np.asarray(z64, np.float64)
    err = np.asarray(z_err, np.float64)
    lo = (z64 - err).astype(np.float32)
    hi = (z64 + err).astype(np.float32)
    return lo, hi


def depth_key_uncertain(z64, z_err):
    """Whether float32(z) could round differently in another float64 evaluation of z."""
    lo, hi = depth_key_range(z64, z_err)
    return lo != hi


def composite_decisions(proj, px, py, s: RenderSettings, rel_margin=1e-5,
                        budget=4_000_000) -> Decisions:
    """Brute force over every valid Gaussian for each pixel: which Gaussians contribute and
    in what order.  Also flags pixels whose result depends on a decision that rounding could
    flip (alpha within rel_margin of alpha_min or alpha_max, T' within rel_margin of t_min, a
    processed Gaussian whose float32 depth key is uncertain (`depth_key_range`) next to
    another processed Gaussian whose key could equal or pass it)."""
    with torch.no_grad():
        vidx = torch.nonzero(proj["valid"]).flatten()
        u = proj["u"][vidx]
        v = proj["v"][vidx]
        A, B, C = proj["conic"][vidx].unbind(-1)
        o = proj["o"][vidx]
        z64 = proj["z"][vidx].numpy()
        zlo, zhi = depth_key_range(z64, proj["z_err"][vidx].numpy())
    z32 = z64.astype(np.float32)
    zunc = zlo != zhi
    vidx_np = vidx.numpy()
    P = len(px)
    lists, clamps, amb, touched = [], [], np.zeros(P, bool), []
    nv = max(1, len(vidx_np))
    chunk = max(1, budget // nv)
    for c0 in range(0, P, chunk):
        c1 = min(P, c0 + chunk)
        cx = torch.tensor(np.asarray(px[c0:c1], np.float64) + 0.5, dtype=DT)[:, None]
        cy = torch.tensor(np.asarray(py[c0:c1], np.float64) + 0.5, dtype=DT)[:, None]
        with torch.no_grad():
            dx = u[None, :] - cx
            dy = v[None, :] - cy
            power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
            araw = o * torch.exp(power)
            alpha = torch.clamp(araw, max=s.alpha_max)
            keep = (power <= 0) & (alpha >= s.alpha_min)
            near_min = (power <= 0) & ((araw - s.alpha_min).abs() <= rel_margin * s.alpha_min)
        keep_np = keep.numpy()
        alpha_np = alpha.numpy()
        araw_np = araw.numpy()
        nearmin_np = near_min.numpy()
        for r in range(c1 - c0):
            k = np.nonzero(keep_np[r])[0]
            order = k[np.lexsort((vidx_np[k], z32[k]))]
            T = 1.0
            out, cl, tch = [], [], []
            ambig = bool(nearmin_np[r].any())
            for j in order:
                a = float(alpha_np[r, j])
                Tn = T * (1.0 - a)
                tch.append(j)
                if abs(araw_np[r, j] - s.alpha_max) <= rel_margin * s.alpha_max:
                    ambig = True
                if abs(Tn - s.t_min) <= rel_margin * s.t_min:
                    ambig = True
                if Tn < s.t_min:
                    break
                out.append(j)
                cl.append(bool(araw_np[r, j] > s.alpha_max))
                T = Tn
            if len(tch) > 1:
                # the order of two processed Gaussians can change only if one's key is
                # uncertain and the other's possible keys meet its range
                ta = np.array(tch)
                for j in ta[zunc[ta]]:
                    others = ta[ta != j]
                    if np.any((zhi[others] >= zlo[j]) & (zlo[others] <= zhi[j])):
                        ambig = True
                        break
            lists.append(vidx_np[np.array(out, dtype=np.int64)] if out else np.zeros(0, np.int64))
            clamps.append(np.array(cl, dtype=bool))
            touched.append(vidx_np[np.array(tch, dtype=np.int64)] if tch else np.zeros(0, np.int64))
            amb[c0 + r] = ambig
    kmax = max([len(l) for l in lists] + [1])
    idx = np.full((P, kmax), -1, np.int64)
    clamped = np.zeros((P, kmax), bool)
    count = np.zeros(P, np.int64)
    for r, (l, cl) in enumerate(zip(lists, clamps)):
        idx[r, :len(l)] = l
        clamped[r, :len(l)] = cl
        count[r] = len(l)
    return Decisions(idx, clamped, count, amb, touched)


def composite_eval(proj, px, py, dec: Decisions, s: RenderSettings):
    """Differentiable compositing of the frozen per-pixel lists (float64)."""
    P, kmax = dec.idx.shape
    idx = torch.tensor(np.where(dec.idx >= 0, dec.idx, 0))
    m = torch.tensor(dec.idx >= 0)
    cx = torch.tensor(np.asarray(px, np.float64) + 0.5, dtype=DT)[:, None]
    cy = torch.tensor(np.asarray(py, np.float64) + 0.5, dtype=DT)[:, None]
    u = proj["u"][idx]
    v = proj["v"][idx]
    con = proj["conic"][idx]
    dx = u - cx
    dy = v - cy
    power = -0.5 * (con[..., 0] * dx * dx + con[..., 2] * dy * dy) - con[..., 1] * dx * dy
    araw = proj["o"][idx] * torch.exp(power)
    alpha = torch.where(torch.tensor(dec.clamped), torch.full_like(araw, s.alpha_max), araw)
    alpha = torch.where(m, alpha, torch.zeros_like(alpha))
    T_after = torch.cumprod(1.0 - alpha, dim=1)
    T_before = torch.cat([torch.ones(P, 1, dtype=DT), T_after[:, :-1]], dim=1)
    w = alpha * T_before
    T_final = T_after[:, -1]
    bg = torch.tensor(s.bg, dtype=DT)
    rgb = (w[..., None] * proj["rgb"][idx]).sum(1) + T_final[:, None] * bg
    z = proj["z"][idx]
    depth = (w * z).sum(1)
    acc = w.sum(1)
    depth2 = (w * z * z).sum(1)
    return rgb, depth, acc, T_final, depth2


def _pixel_coords(cam, pix):
    pix = np.asarray(pix, np.int64)
    return pix % cam.width, pix // cam.width


def render(scene, s: RenderSettings = None, pixels=None, p=None):
    """Forward render.  `pixels`: per view flat pixel indices (y * W + x), or None for full
    images.  Returns per view dict(rgb (P,3), depth, alpha, T, count, ambiguous, pix)."""
    s = s or RenderSettings()
    p = p if p is not None else leaves(scene, requires_grad=False)
    out = []
    with torch.no_grad():
        for b, cam in enumerate(scene.cameras):
            pix = np.arange(cam.width * cam.height) if pixels is None or pixels[b] is None \
                else np.asarray(pixels[b], np.int64)
            px, py = _pixel_coords(cam, pix)
            proj = project(p, cam, p["pose_delta"][b], s, scene.sh_degree)
            dec = composite_decisions(proj, px, py, s)
            rgb, depth, acc, T, depth2 = composite_eval(proj, px, py, dec, s)
            out.append({"rgb": rgb.numpy(), "depth": depth.numpy(), "alpha": acc.numpy(),
                        "depth2": depth2.numpy(),
                        "T": T.numpy(), "count": dec.count, "ambiguous": dec.ambiguous,
                        "pix": pix, "proj": proj, "dec": dec})
    return out


def _dilate(cam, pix, r):
    """Pixels within Chebyshev distance r of `pix` (flat indices), inside the image."""
    img = np.zeros((cam.height, cam.width), bool)
    px, py = _pixel_coords(cam, pix)
    img[py, px] = True
    out = np.zeros_like(img)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            ys = slice(max(0, dy), cam.height + min(0, dy))
            yd = slice(max(0, -dy), cam.height + min(0, -dy))
            xs = slice(max(0, dx), cam.width + min(0, dx))
            xd = slice(max(0, -dx), cam.width + min(0, -dx))
            out[yd, xd] |= img[ys, xs]
    return np.flatnonzero(out.ravel())


def loss_and_grads(scene, s: RenderSettings = None, masks=None, lidar=None, gt=None,
                   w_l1: float = 1.0, lam: float = 1.0, upstream=None, sign_margin=1e-5,
                   frozen=None, deltas=None, ssim_w: float = 0.0, sigma_mode: str = "fixed",
                   sigma_floor: float = 1e-4, stats: bool = False):
    """Loss of Sec. III-C (L1 and D-SSIM parts of L_3DGS + LiDAR KL term) and its float64
    gradients.

    masks: per view flat pixel indices where the L1 term applies (None = whole image).
    lidar: per view dict(pix, depth, sigma) (defaults to scene.lidar); its pixels are
           always evaluated.
    upstream: optional per view dict(rgb (3,H,W), depth (H,W), alpha (H,W)) -- then the
           objective is sum(upstream * outputs) over whole images instead of the loss.
    frozen: decisions from a previous call (to evaluate the same piecewise-smooth branch).
    Returns dict(loss, grads{name: np}, pose (B,6), views[...], amb_gauss (N,) bool,
    decisions).
    """
    s = s or RenderSettings()
    lidar = scene.lidar if lidar is None else lidar
    gt = scene.gt_rgb if gt is None else gt
    p = leaves(scene, requires_grad=True, deltas=deltas)
    total = torch.zeros((), dtype=DT)
    views = []
    amb_gauss = np.zeros(scene.n, bool)
    decisions = []
    projs = []
    for b, cam in enumerate(scene.cameras):
        HW = cam.width * cam.height
        if upstream is not None:
            eval_pix = np.arange(HW)
            l1_pix = None
        else:
            l1_pix = np.arange(HW) if masks is None or masks[b] is None else np.asarray(masks[b], np.int64)
            lp = np.asarray(lidar[b]["pix"], np.int64) if lidar and len(lidar[b]["pix"]) else np.zeros(0, np.int64)
            eval_pix = np.union1d(l1_pix, lp)
            if ssim_w > 0.0:  # the SSIM windows of the mask pixels
                eval_pix = np.union1d(eval_pix, _dilate(cam, l1_pix, window_radius()))
        px, py = _pixel_coords(cam, eval_pix)
        proj = project(p, cam, p["pose_delta"][b], s, scene.sh_degree)
        if stats:
            proj["u"].retain_grad()
            proj["v"].retain_grad()
            projs.append(proj)
        if frozen is not None:
            dec = frozen[b]
        else:
            dec = composite_decisions(proj, px, py, s)
        decisions.append(dec)
        rgb, depth, acc, T, depth2 = composite_eval(proj, px, py, dec, s)
        pos = {int(q): k for k, q in enumerate(eval_pix)}
        amb_pix = dec.ambiguous.copy()
        if upstream is not None:
            up = upstream[b]
            g_rgb = torch.tensor(np.asarray(up["rgb"], np.float64).reshape(3, -1).T[eval_pix])
            g_d = torch.tensor(np.asarray(up["depth"], np.float64).reshape(-1)[eval_pix])
            g_a = torch.tensor(np.asarray(up["alpha"], np.float64).reshape(-1)[eval_pix])
            total = total + (g_rgb * rgb).sum() + (g_d * depth).sum() + (g_a * acc).sum()
        else:
            sel = torch.tensor([pos[int(q)] for q in l1_pix], dtype=torch.long)
            if len(l1_pix):
                tgt = torch.tensor(np.asarray(gt[b], np.float64).reshape(3, -1).T[l1_pix])
                diff = rgb[sel] - tgt
                if frozen is not None and dec.l1_sign is not None and dec.l1_sign.shape == tuple(diff.shape):
                    l1 = (diff * torch.tensor(dec.l1_sign, dtype=DT)).sum()  # the frozen branch of |.|
                else:
                    l1 = diff.abs().sum()
                    dec.l1_sign = np.sign(diff.detach().numpy())
                total = total + (1.0 - ssim_w) * w_l1 / (3.0 * len(l1_pix)) * l1
                close = (diff.detach().abs() < sign_margin).any(1).numpy()
                amb_pix[sel.numpy()[close]] = True
                if ssim_w > 0.0:
                    img = torch.zeros(3, cam.height * cam.width, dtype=DT)
                    img[:, torch.tensor(eval_pix)] = rgb.T
                    smap = ssim_map(img.view(3, cam.height, cam.width),
                                    torch.tensor(np.asarray(gt[b], np.float64)))
                    s_sel = smap.reshape(3, -1)[:, torch.tensor(l1_pix)]
                    total = total + ssim_w * w_l1 / (3.0 * len(l1_pix)) * (1.0 - s_sel).sum()
            if lidar and len(lidar[b]["pix"]):
                li = torch.tensor([pos[int(q)] for q in lidar[b]["pix"]], dtype=torch.long)
                dl = torch.tensor(np.asarray(lidar[b]["depth"], np.float64))
                sl = torch.tensor(np.asarray(lidar[b]["sigma"], np.float64))
                mu_u = depth[li]
                if sigma_mode == "rendered":
                    # sigma_u^2 = sum w z^2 - mu_u^2 + floor (the rendered depth variance)
                    su = torch.sqrt(depth2[li] - mu_u * mu_u + sigma_floor)
                else:
                    su = sl
                kl = kl_normal(dl, sl, mu_u, su)
                total = total + lam / len(li) * kl.sum()
        for r in np.nonzero(amb_pix)[0]:
            amb_gauss[cam.g_begin + dec.touched[r]] = True
        views.append({"rgb": rgb.detach().numpy(), "depth": depth.detach().numpy(),
                      "alpha": acc.detach().numpy(), "T": T.detach().numpy(),
                      "count": dec.count, "ambiguous": amb_pix, "pix": eval_pix})
    total.backward()
    grads = {k: (v.grad.numpy().copy() if v.grad is not None else np.zeros(v.shape))
             for k, v in p.items()}
    pose = grads.pop("pose_delta")
    out = {"loss": float(total.detach()), "grads": grads, "pose": pose, "views": views,
           "amb_gauss": amb_gauss, "decisions": decisions}
    if stats:
        out["stats"] = image_gradient_stats(scene, projs)
    return out


def image_gradient_stats(scene, projs, margin=1e-4):
    """Densification statistics (Sec. III-B, lifecycle operations: the image-space gradient
    magnitude at the projected splat centre): per Gaussian, the sum over the views that see
    it of |dL/d(u, v)| (pixel units) and the number of those views.  A view sees a Gaussian
    when it survives culling and its footprint rectangle meets the image; `ambiguous` marks
    Gaussians whose rectangle edge lies within `margin` px of flipping that test."""
    n = scene.n
    acc = np.zeros(n)
    cnt = np.zeros(n, np.int64)
    amb = np.zeros(n, bool)
    for cam, proj in zip(scene.cameras, projs):
        g0 = proj["g0"]
        gu = proj["u"].grad
        gv = proj["v"].grad
        gu = np.zeros(len(proj["u"])) if gu is None else gu.numpy()
        gv = np.zeros(len(proj["v"])) if gv is None else gv.numpy()
        u = proj["u"].detach().numpy()
        v = proj["v"].detach().numpy()
        ex, ey = proj["ext"][:, 0].numpy(), proj["ext"][:, 1].numpy()
        valid = proj["valid"].numpy()
        lo_x, hi_x = u - ex - 0.5, u + ex - 0.5
        lo_y, hi_y = v - ey - 0.5, v + ey - 0.5
        x0, x1 = np.clip(np.floor(lo_x), 0, cam.width), np.clip(np.ceil(hi_x), -1, cam.width - 1)
        y0, y1 = np.clip(np.floor(lo_y), 0, cam.height), np.clip(np.ceil(hi_y), -1, cam.height - 1)
        seen = valid & (x0 <= x1) & (y0 <= y1)
        near = lambda t: np.abs(t - np.round(t)) < margin
        edge = (near(hi_x) & (np.abs(np.ceil(hi_x)) <= 1)) | (near(lo_x) & (np.abs(np.floor(lo_x) - cam.width) <= 1)) | \
               (near(hi_y) & (np.abs(np.ceil(hi_y)) <= 1)) | (near(lo_y) & (np.abs(np.floor(lo_y) - cam.height) <= 1))
        idx = np.arange(g0, g0 + len(u))
        acc[idx] += np.where(seen, np.hypot(gu, gv), 0.0)
        cnt[idx] += seen
        amb[idx] |= valid & edge
    return {"grad_accum": acc, "count": cnt, "ambiguous": amb}


def frozen_objective(scene, decisions, s: RenderSettings = None, masks=None, lidar=None,
                     gt=None, w_l1=1.0, lam=1.0, upstream=None, deltas=None, ssim_w=0.0,
                     sigma_mode="fixed", sigma_floor=1e-4):
    """The same objective as `loss_and_grads` evaluated with given frozen decisions and no
    gradient (used by finite differences)."""
    s = s or RenderSettings()
    with torch.enable_grad():
        r = loss_and_grads(scene, s, masks, lidar, gt, w_l1, lam, upstream, frozen=decisions,
                           deltas=deltas, ssim_w=ssim_w, sigma_mode=sigma_mode, sigma_floor=sigma_floor)
    return r["loss"]
