"""Pins for the oracle's rotations, covariances, SE(3) maps and spherical harmonics.

Covariance: Sec. III-B (Sigma = R S S^T R^T).  SE(3): the Exp map of the paper's motion
model (Sec. III-A) reused for the left pose perturbation.  SH: the per-splat colour
coefficients of Sec. III-B under the real, Condon-Shortley-phase reading.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.special
import torch

from oracle.geometry import covariance_3d, quat_to_rotmat, se3_exp, se3_exp_torch, skew
from oracle.sh import real_sh

DT = torch.float64


def test_identity_quaternion_gives_axis_aligned_covariance():
    s = torch.tensor([[-1.0, -2.0, 0.5]], dtype=DT)
    q = torch.tensor([[1.0, 0, 0, 0]], dtype=DT)
    S = covariance_3d(s, q)[0].numpy()
    assert np.allclose(S, np.diag(np.exp(2 * s[0].numpy())), atol=1e-15)


def test_quarter_turn_about_z_swaps_x_and_y_variances():
    s = torch.tensor([[-1.0, -2.0, 0.5]], dtype=DT)
    h = math.sqrt(0.5)
    q = torch.tensor([[h, 0, 0, h]], dtype=DT)  # 90 deg about z
    S = covariance_3d(s, q)[0].numpy()
    e = np.exp(2 * s[0].numpy())
    assert np.allclose(np.diag(S), [e[1], e[0], e[2]], atol=1e-14)
    R = quat_to_rotmat(q)[0].numpy()
    assert np.allclose(R @ np.array([1.0, 0, 0]), [0, 1, 0], atol=1e-15)


def test_rotation_matches_axis_angle_exponential_and_quaternion_scale_is_ignored():
    rng = np.random.default_rng(0)
    for _ in range(20):
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        ang = rng.uniform(-math.pi, math.pi)
        q = np.r_[math.cos(ang / 2), math.sin(ang / 2) * axis] * rng.uniform(0.2, 5)
        R = quat_to_rotmat(torch.tensor(q[None], dtype=DT))[0].numpy()
        assert np.allclose(R, scipy.linalg.expm(ang * skew(axis)), atol=1e-13)


def test_covariance_is_symmetric_positive_definite():
    rng = np.random.default_rng(1)
    s = torch.tensor(rng.normal(-2, 1, (50, 3)), dtype=DT)
    q = torch.tensor(rng.normal(size=(50, 4)), dtype=DT)
    S = covariance_3d(s, q).numpy()
    assert np.allclose(S, S.transpose(0, 2, 1), atol=1e-15)
    ev = np.linalg.eigvalsh(S)
    assert (ev > 0).all()
    # eigenvalues are the squared scales
    assert np.allclose(np.sort(ev, 1), np.sort(np.exp(2 * s.numpy()), 1), rtol=1e-10)


def _twist(delta):
    X = np.zeros((4, 4))
    X[:3, :3] = skew(delta[3:])
    X[:3, 3] = delta[:3]
    return X


@pytest.mark.parametrize("scale", [0.0, 1e-9, 1e-5, 1e-3, 0.3, 2.5])
def test_se3_exp_matches_matrix_exponential(scale):
    rng = np.random.default_rng(2)
    for _ in range(5):
        d = rng.normal(size=6) * scale
        E = se3_exp(d)
        assert np.allclose(E, scipy.linalg.expm(_twist(d)), atol=1e-13)
        # inverse
        assert np.allclose(E @ se3_exp(-d), np.eye(4), atol=1e-13)
        Rt, tt = se3_exp_torch(torch.tensor(d, dtype=DT))
        assert np.allclose(Rt.numpy(), E[:3, :3], atol=1e-13)
        assert np.allclose(tt.numpy(), E[:3, 3], atol=1e-13)


def test_se3_exp_of_zero_is_identity_and_derivative_is_the_hat_map():
    assert np.array_equal(se3_exp(np.zeros(6)), np.eye(4))
    # d/d delta_j Exp(delta) at 0 equals the generator G_j (central FD of the closed form)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        D = (se3_exp(e) - se3_exp(-e)) / (2 * h)
        G = np.zeros(6)
        G[j] = 1
        assert np.allclose(D, _twist(G), atol=1e-9)


# ------------------------------------------------------------------ spherical harmonics
def _scipy_real_sh(lmax, dirs):
    """Real SH built from scipy's complex Y_l^m (which includes the Condon-Shortley
    phase): Y_lm = sqrt2 Re Y_l^m (m>0), sqrt2 Im Y_l^|m| (m<0), Y_l^0 (m=0)."""
    x, y, z = dirs.T
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    cols = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                cols.append(Y.real)
            elif m > 0:
                cols.append(math.sqrt(2) * Y.real)
            else:
                cols.append(math.sqrt(2) * Y.imag)
    return np.stack(cols, -1)


def test_real_sh_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(3)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ours = real_sh(3, torch.tensor(d, dtype=DT)).numpy()
    assert np.allclose(ours, _scipy_real_sh(3, d), atol=1e-12)


def test_real_sh_is_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform trapezoid in phi: exact for these degrees
    nt, nphi = 16, 32
    ct, wt = np.polynomial.legendre.leggauss(nt)
    phi = 2 * math.pi * np.arange(nphi) / nphi
    C, P = np.meshgrid(ct, phi, indexing="ij")
    st = np.sqrt(1 - C ** 2)
    dirs = np.stack([st * np.cos(P), st * np.sin(P), C], -1).reshape(-1, 3)
    w = (wt[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y = real_sh(3, torch.tensor(dirs, dtype=DT)).numpy()
    G = (Y * w[:, None]).T @ Y
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_real_sh_low_degree_closed_forms():
    """Fixes the sign convention: Y_00 = 1/(2 sqrt pi); degree 1 is
    sqrt(3/(4 pi)) * (-y, z, -x) for m = -1, 0, 1 (Condon-Shortley phase)."""
    rng = np.random.default_rng(4)
    d = rng.normal(size=(10, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = real_sh(1, torch.tensor(d, dtype=DT)).numpy()
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 0], c0, atol=1e-15)
    assert np.allclose(Y[:, 1], -c1 * d[:, 1], atol=1e-15)
    assert np.allclose(Y[:, 2], c1 * d[:, 2], atol=1e-15)
    assert np.allclose(Y[:, 3], -c1 * d[:, 0], atol=1e-15)
