"""Rotations, covariances and SE(3) maps in float64 (oracle; test infrastructure only).

* quaternion -> rotation: the standard unit-quaternion matrix (w first), after normalising q.
* 3D covariance Sigma = R S S^T R^T with S = diag(exp(log_scale))   (Sec. III-B).
* SE(3) exponential of a twist delta = (rho, phi), translation first: rotation by
  Rodrigues' formula, translation V rho with V the left Jacobian of SO(3).  Used for the
  left-perturbation pose model W <- Exp(delta) W (poses refined through the projection,
  Sec. III-C) and for the retraction after an optimiser step.
"""
from __future__ import annotations

import math

import numpy as np
import torch

DT = torch.float64


def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """(N, 4) wxyz quaternions (any norm) -> (N, 3, 3) rotation matrices."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    rows = [
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ]
    return torch.stack(rows, -2)


def covariance_3d(log_scales: torch.Tensor, quats: torch.Tensor) -> torch.Tensor:
    """Sigma = R S S^T R^T, S = diag(exp(s))  (Sec. III-B covariance equation)."""
    R = quat_to_rotmat(quats)
    M = R * torch.exp(log_scales)[..., None, :]  # R @ diag(e^s)
    return M @ M.transpose(-1, -2)


def skew(v):
    """[v]_x such that [v]_x w = v x w (numpy or torch, last dim 3)."""
    if isinstance(v, torch.Tensor):
        z = torch.zeros_like(v[..., 0])
        return torch.stack([torch.stack([z, -v[..., 2], v[..., 1]], -1),
                            torch.stack([v[..., 2], z, -v[..., 0]], -1),
                            torch.stack([-v[..., 1], v[..., 0], z], -1)], -2)
    v = np.asarray(v, dtype=np.float64)
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def se3_exp(delta) -> np.ndarray:
    """4x4 homogeneous Exp(delta), delta = (rho, phi) in float64 (closed form)."""
    delta = np.asarray(delta, dtype=np.float64)
    rho, phi = delta[:3], delta[3:]
    th = float(np.linalg.norm(phi))
    K = skew(phi)
    if th < 1e-4:
        # Taylor expansions of sin(t)/t, (1-cos t)/t^2, (t - sin t)/t^3 around 0
        a = 1 - th ** 2 / 6 + th ** 4 / 120
        b = 0.5 - th ** 2 / 24 + th ** 4 / 720
        c = 1.0 / 6 - th ** 2 / 120 + th ** 4 / 5040
    else:
        a = math.sin(th) / th
        b = (1 - math.cos(th)) / th ** 2
        c = (th - math.sin(th)) / th ** 3
    R = np.eye(3) + a * K + b * (K @ K)
    V = np.eye(3) + b * K + c * (K @ K)
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def se3_exp_torch(delta: torch.Tensor):
    """Differentiable Exp for autograd: returns (R (3,3), t (3,)).  Uses the series in
    theta^2 (no square root) so the derivative at delta = 0 is exact."""
    rho, phi = delta[:3], delta[3:]
    th2 = (phi * phi).sum()
    K = skew(phi)
    if float(th2.detach()) < 1e-8:
        a = 1 - th2 / 6 + th2 * th2 / 120
        b = 0.5 - th2 / 24 + th2 * th2 / 720
        c = 1.0 / 6 - th2 / 120 + th2 * th2 / 5040
    else:
        th = torch.sqrt(th2)
        a = torch.sin(th) / th
        b = (1 - torch.cos(th)) / th2
        c = (th - torch.sin(th)) / (th2 * th)
    eye = torch.eye(3, dtype=delta.dtype)
    R = eye + a * K + b * (K @ K)
    V = eye + b * K + c * (K @ K)
    return R, V @ rho


def perturb_pose(R: np.ndarray, t: np.ndarray, delta) -> tuple[np.ndarray, np.ndarray]:
    """Left perturbation W <- Exp(delta) W of a world->camera pose (float64)."""
    E = se3_exp(delta)
    R64 = np.asarray(R, np.float64)
    t64 = np.asarray(t, np.float64)
    return E[:3, :3] @ R64, E[:3, :3] @ t64 + E[:3, 3]
