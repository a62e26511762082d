"""Structural similarity of a rendered image and its target, for the D-SSIM part of the
photometric loss (oracle; tests only).

The photometric loss of Sec. III-C is L_3DGS = (1 - lambda) L1 + lambda L_D-SSIM, the loss of
standard 3DGS.  The paper gives neither lambda nor the SSIM constants; the readings taken
here are the usual ones:
    L_D-SSIM = 1 - SSIM, SSIM the mean over pixels and colour channels of the SSIM map
    s = ((2 mu_x mu_y + C1)(2 sigma_xy + C2)) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)),
with local statistics weighted by an 11 x 11 Gaussian window (sigma 1.5, normalised to sum 1),
the image padded with zeros (output the size of the input), C1 = 0.01^2, C2 = 0.03^2
(dynamic range 1), each channel on its own:
    mu_x = G * x, sigma_x^2 = G * x^2 - mu_x^2, sigma_xy = G * (x y) - mu_x mu_y.
Written from that definition in float64 torch (differentiable).
"""
from __future__ import annotations

import torch

DT = torch.float64
C1 = 0.01 ** 2
C2 = 0.03 ** 2


def gaussian_window(size: int = 11, sigma: float = 1.5) -> torch.Tensor:
    """1D Gaussian weights at integer offsets -size//2 .. size//2, normalised to sum 1."""
    r = size // 2
    k = torch.arange(-r, r + 1, dtype=DT)
    w = torch.exp(-k * k / (2.0 * sigma * sigma))
    return w / w.sum()


def blur(img: torch.Tensor, size: int = 11, sigma: float = 1.5) -> torch.Tensor:
    """Zero-padded Gaussian-weighted local mean of each channel of img (..., H, W): the 2D
    window is the outer product of the 1D weights, applied as a row pass then a column
    pass."""
    w = gaussian_window(size, sigma)
    r = size // 2
    H, W = img.shape[-2], img.shape[-1]
    pad = torch.nn.functional.pad(img, (r, r, r, r))
    rows = sum(w[k] * pad[..., :, k:k + W] for k in range(size))        # (..., H + 2r, W)
    return sum(w[k] * rows[..., k:k + H, :] for k in range(size))       # (..., H, W)


def ssim_map(x: torch.Tensor, y: torch.Tensor, size: int = 11, sigma: float = 1.5) -> torch.Tensor:
    """Per-pixel, per-channel SSIM of x against y, both (C, H, W)."""
    mx, my = blur(x, size, sigma), blur(y, size, sigma)
    sxx = blur(x * x, size, sigma) - mx * mx
    syy = blur(y * y, size, sigma) - my * my
    sxy = blur(x * y, size, sigma) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def window_radius(size: int = 11) -> int:
    return size // 2
