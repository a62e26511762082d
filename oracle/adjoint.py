"""Hand-derived float64 adjoint of projection and compositing (oracle; tests only).

A second statement of the gradients of `oracle.render`, written out with the chain rule
instead of autograd, for the objective sum_b sum_p (g_C . C + g_D D + g_A A) with given
upstream images (Sec. III-B compositing and projection, Sec. III-C pose refinement through
the projection).  Per pixel, contributors k = 1..n in composite order, T_1 = 1,
T_{k+1} = T_k (1 - alpha_k), w_k = alpha_k T_k:
    dC/dc_k = w_k,  dD/dz_k = w_k,
    g_alpha_k = T_k (g_C.c_k + g_D z_k + g_A)
                - (g_C.S^C_k + g_D S^D_k + g_A S^A_k + T_{n+1} g_C.bg) / (1 - alpha_k)
with the suffix sums S^F_k = sum_{j > k} w_j F_j; where alpha is not clamped,
alpha = o e^power gives g_o = g_alpha e^power and g_power = g_alpha alpha, and power =
-(a dx^2 + c dy^2)/2 - b dx dy (dx = u - pixel centre) passes it to (u, v) and the conic.
Projection: G_Sigma' = -K G_K K (K the conic), Sigma' = J Sigma_c J^T, Sigma_c = R_b Sigma
R_b^T, Sigma = M M^T with M = R(q) diag(e^s); J depends on the camera-frame mean (through
the field-of-view clamp where it is active); the colour max(0, Y(d).f + 1/2) depends on the
unit direction d from the camera centre; the pose perturbation is the left one,
W_b <- Exp(delta) W_b, delta = (rho, phi), at delta = 0.
Discrete decisions (kept sets, order, stop, clamps) are those of the forward (`Decisions`).
The SH basis gradient comes from complex-step differentiation of the basis polynomials.
"""
from __future__ import annotations

import numpy as np
import torch

from .geometry import skew
from .render import _pixel_coords, composite_decisions, leaves, project
from .settings import RenderSettings
from .sh import real_sh


def _sh_and_grad(deg, d):
    """Y(d) (n, K) and dY/dd (n, K, 3) by complex-step differentiation (exact for the
    polynomial basis up to rounding)."""
    Y = real_sh(deg, torch.tensor(d)).numpy()
    h = 1e-30
    G = np.zeros(Y.shape + (3,))
    for c in range(3):
        dc = d.astype(np.complex128)
        dc[:, c] += 1j * h
        Yc = real_sh(deg, torch.tensor(dc)).numpy()
        G[..., c] = Yc.imag / h
    return Y, G


def _quat_rot(qn):
    w, x, y, z = qn
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _quat_rot_grad(qn):
    """dR/dw, dR/dx, dR/dy, dR/dz of the unit-quaternion rotation matrix."""
    w, x, y, z = qn
    return np.array([
        [[0, -2 * z, 2 * y], [2 * z, 0, -2 * x], [-2 * y, 2 * x, 0]],
        [[0, 2 * y, 2 * z], [2 * y, -4 * x, -2 * w], [2 * z, 2 * w, -4 * x]],
        [[-4 * y, 2 * x, 2 * w], [2 * x, 0, 2 * z], [-2 * w, 2 * z, -4 * y]],
        [[-4 * z, -2 * w, 2 * x], [2 * w, -4 * z, 2 * y], [2 * x, 2 * y, 0]]], np.float64)


def upstream_grads(scene, upstream, s: RenderSettings = None, decisions=None):
    """Gradients of sum_b sum_p (g_C.C + g_D D + g_A A) (upstream[b] = dict(rgb (3,H,W),
    depth (H,W), alpha (H,W))) at the scene's parameters and poses.  Returns dict(grads{name:
    (N, ...)}, pose (B, 6))."""
    s = s or RenderSettings()
    N = scene.n
    deg = scene.sh_degree
    K = (deg + 1) ** 2
    means = np.asarray(scene.means, np.float64)
    ls = np.asarray(scene.log_scales, np.float64)
    quats = np.asarray(scene.quats, np.float64)
    logits = np.asarray(scene.opacity_logits, np.float64)
    sh = np.asarray(scene.sh, np.float64)
    g = {"means": np.zeros((N, 3)), "log_scales": np.zeros((N, 3)), "quats": np.zeros((N, 4)),
         "opacity_logits": np.zeros(N), "sh": np.zeros((N, K, 3))}
    pose = np.zeros((len(scene.cameras), 6))
    bg = np.asarray(s.bg, np.float64)
    p_leaf = leaves(scene, requires_grad=False) if decisions is None else None
    for b, cam in enumerate(scene.cameras):
        g0, g1 = cam.g_begin, cam.g_end
        n = g1 - g0
        R = np.asarray(cam.R, np.float64)
        t = np.asarray(cam.t, np.float64)
        # ---- forward, per Gaussian of the view
        mu = means[g0:g1]
        xc = mu @ R.T + t
        x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
        valid = z >= s.z_near
        zs = np.where(valid, z, 1.0)
        limx = s.fov_clamp * cam.width / (2.0 * cam.fx)
        limy = s.fov_clamp * cam.height / (2.0 * cam.fy)
        rx, ry = x / zs, y / zs
        clx = (rx < -limx) | (rx > limx)
        cly = (ry < -limy) | (ry > limy)
        cxr, cyr = np.clip(rx, -limx, limx), np.clip(ry, -limy, limy)
        J = np.zeros((n, 2, 3))
        J[:, 0, 0] = cam.fx / zs
        J[:, 0, 2] = -cam.fx * cxr / zs
        J[:, 1, 1] = cam.fy / zs
        J[:, 1, 2] = -cam.fy * cyr / zs
        qn = quats[g0:g1] / np.linalg.norm(quats[g0:g1], axis=1, keepdims=True)
        Rq = np.stack([_quat_rot(q) for q in qn])
        es = np.exp(ls[g0:g1])
        M = Rq * es[:, None, :]
        Sig = M @ M.transpose(0, 2, 1)
        Sc = R @ Sig @ R.T
        S2 = J @ Sc @ J.transpose(0, 2, 1) + s.blur * np.eye(2)
        det = S2[:, 0, 0] * S2[:, 1, 1] - S2[:, 0, 1] ** 2
        valid &= det > 0
        dets = np.where(valid, det, 1.0)
        ca, cb, cc = S2[:, 1, 1] / dets, -S2[:, 0, 1] / dets, S2[:, 0, 0] / dets
        u = cam.fx * x / zs + cam.cx
        v = cam.fy * y / zs + cam.cy
        o = 1.0 / (1.0 + np.exp(-logits[g0:g1]))
        valid &= o >= s.alpha_min
        C0 = -(R.T @ t)
        dv = mu - C0
        dist = np.linalg.norm(dv, axis=1)
        d = dv / dist[:, None]
        Y, dY = _sh_and_grad(deg, d)
        raw = np.einsum("nk,nkc->nc", Y, sh[g0:g1]) + 0.5
        rgb = np.maximum(raw, 0.0)
        # ---- per pixel, with the forward's decisions
        HW = cam.width * cam.height
        pix = np.arange(HW)
        px, py = _pixel_coords(cam, pix)
        if decisions is None:
            proj = project(p_leaf, cam, p_leaf["pose_delta"][b], s, deg)
            dec = composite_decisions(proj, px, py, s)
        else:
            dec = decisions[b]
        up = upstream[b]
        gC = np.asarray(up["rgb"], np.float64).reshape(3, -1).T
        gD = np.asarray(up["depth"], np.float64).reshape(-1)
        gA = np.asarray(up["alpha"], np.float64).reshape(-1)
        idx = dec.idx
        live = idx >= 0
        ii = np.where(live, idx, 0)
        cxp = (px + 0.5)[:, None]
        cyp = (py + 0.5)[:, None]
        dx = u[ii] - cxp
        dy = v[ii] - cyp
        pw = -0.5 * (ca[ii] * dx * dx + cc[ii] * dy * dy) - cb[ii] * dx * dy
        G = np.exp(pw)
        alpha = np.where(dec.clamped, s.alpha_max, o[ii] * G)
        alpha = np.where(live, alpha, 0.0)
        Tb = np.cumprod(np.concatenate([np.ones((len(pix), 1)), 1.0 - alpha], 1), 1)
        T_before, T_final = Tb[:, :-1], Tb[:, -1]
        w = alpha * T_before
        col = rgb[ii]                     # (P, Kmax, 3)
        zz = z[ii]

        def suffix(f):                    # sum_{j > k} w_j f_j
            c = np.cumsum((w * f)[:, ::-1], 1)[:, ::-1]
            return c - w * f

        SC = np.stack([suffix(col[..., c]) for c in range(3)], -1)
        SD = suffix(zz)
        SA = suffix(np.ones_like(w))
        own = (col * gC[:, None, :]).sum(-1) + gD[:, None] * zz + gA[:, None]
        later = (SC * gC[:, None, :]).sum(-1) + gD[:, None] * SD + gA[:, None] * SA \
            + T_final[:, None] * (gC @ bg)[:, None]
        g_alpha = np.where(live, T_before * own - later / (1.0 - alpha), 0.0)
        free = live & ~dec.clamped
        g_o_pix = np.where(free, g_alpha * G, 0.0)
        g_pw = np.where(free, g_alpha * alpha, 0.0)
        # scatter to the Gaussians of the view
        gu = np.zeros(n)
        gv = np.zeros(n)
        gcon = np.zeros((n, 3))
        go = np.zeros(n)
        gcol = np.zeros((n, 3))
        gz = np.zeros(n)
        li = ii[live]
        np.add.at(gu, li, (-g_pw * (ca[ii] * dx + cb[ii] * dy))[live])
        np.add.at(gv, li, (-g_pw * (cb[ii] * dx + cc[ii] * dy))[live])
        np.add.at(gcon[:, 0], li, (-0.5 * dx * dx * g_pw)[live])
        np.add.at(gcon[:, 1], li, (-dx * dy * g_pw)[live])
        np.add.at(gcon[:, 2], li, (-0.5 * dy * dy * g_pw)[live])
        np.add.at(go, li, g_o_pix[live])
        for c in range(3):
            np.add.at(gcol[:, c], li, (w * gC[:, None, c])[live])
        np.add.at(gz, li, (w * gD[:, None])[live])
        # ---- projection backward, per Gaussian of the view
        for i in np.nonzero(valid)[0]:
            Kc = np.array([[ca[i], cb[i]], [cb[i], cc[i]]])
            GK = np.array([[gcon[i, 0], 0.5 * gcon[i, 1]], [0.5 * gcon[i, 1], gcon[i, 2]]])
            GS2 = -Kc @ GK @ Kc
            Ji = J[i]
            GSc = Ji.T @ GS2 @ Ji
            GJ = 2.0 * GS2 @ Ji @ Sc[i]
            gx = np.zeros(3)
            # (u, v) = (fx x / z + cx, fy y / z + cy)
            gx[0] += gu[i] * cam.fx / zs[i]
            gx[2] += -gu[i] * cam.fx * x[i] / zs[i] ** 2
            gx[1] += gv[i] * cam.fy / zs[i]
            gx[2] += -gv[i] * cam.fy * y[i] / zs[i] ** 2
            gx[2] += gz[i]
            # J(x_c): J00 = fx / z, J11 = fy / z, J02 = -fx r_x / z with r_x = clamp(x / z)
            gx[2] += GJ[0, 0] * (-cam.fx / zs[i] ** 2) + GJ[1, 1] * (-cam.fy / zs[i] ** 2)
            if clx[i]:
                gx[2] += GJ[0, 2] * cam.fx * cxr[i] / zs[i] ** 2
            else:
                gx[0] += GJ[0, 2] * (-cam.fx / zs[i] ** 2)
                gx[2] += GJ[0, 2] * 2.0 * cam.fx * x[i] / zs[i] ** 3
            if cly[i]:
                gx[2] += GJ[1, 2] * cam.fy * cyr[i] / zs[i] ** 2
            else:
                gx[1] += GJ[1, 2] * (-cam.fy / zs[i] ** 2)
                gx[2] += GJ[1, 2] * 2.0 * cam.fy * y[i] / zs[i] ** 3
            GSig = R.T @ GSc @ R
            GM = (GSig + GSig.T) @ M[i]
            gi = g0 + i
            g["log_scales"][gi] += np.einsum("rj,rj->j", GM, M[i])
            GR = GM * es[i][None, :]
            gqn = np.einsum("rc,krc->k", GR, _quat_rot_grad(qn[i]))
            qnorm = np.linalg.norm(quats[gi])
            g["quats"][gi] += (gqn - qn[i] * (qn[i] @ gqn)) / qnorm
            g["opacity_logits"][gi] += go[i] * o[i] * (1.0 - o[i])
            graw = np.where(raw[i] > 0.0, gcol[i], 0.0)
            g["sh"][gi] += Y[i][:, None] * graw[None, :]
            gd = np.einsum("kc,c,kj->j", sh[gi], graw, dY[i])
            gmu_sh = (gd - d[i] * (d[i] @ gd)) / dist[i]
            g["means"][gi] += R.T @ gx + gmu_sh
            # pose: x_c' = x_c + phi x x_c + rho, Sigma_c' = Sigma_c + [phi]x Sigma_c - Sigma_c [phi]x,
            # camera centre C' = C - R^T rho (first order)
            pose[b, :3] += gx + R @ gmu_sh
            pose[b, 3:] += np.cross(xc[i], gx)
            for k in range(3):
                E = skew(np.eye(3)[k])
                pose[b, 3 + k] += np.sum(GSc * (E @ Sc[i] - Sc[i] @ E))
    return {"grads": g, "pose": pose}
