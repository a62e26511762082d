"""Real spherical harmonics up to degree 3, differentiable, float64 (oracle).

The paper stores a per-splat SH colour vector c in R^{d_SH} (Sec. III-B) without fixing a
convention.  Reading used throughout: orthonormal real SH with the Condon-Shortley phase,
coefficients l-major with m = -l..l,
    Y_l0            = K_l0 P_l^0(z)
    Y_lm  (m > 0)   = sqrt(2) K_lm P_l^m(cos th) cos(m ph)
    Y_l-m (m > 0)   = sqrt(2) K_lm P_l^m(cos th) sin(m ph)
with K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m the associated Legendre function
including (-1)^m.  Written through the standard three-term Legendre recurrence in z and
the powers (x + i y)^m = sin^m(th) e^{i m ph}, so it is a polynomial in the unit
direction (x, y, z) and torch can differentiate it.  Pinned against scipy's complex
spherical harmonics and by quadrature orthonormality in tests/test_oracle_sh.py.
"""
from __future__ import annotations

import math

import torch


def _legendre_reduced(lmax: int, z: torch.Tensor):
    """P_l^m(z) / (1 - z^2)^{m/2} for 0 <= m <= l <= lmax (Condon-Shortley phase included):
    a polynomial in z.  Returns dict (l, m) -> tensor."""
    P = {}
    for m in range(lmax + 1):
        # P_m^m / sin^m = (-1)^m (2m-1)!!
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        pmm = torch.full_like(z, ((-1.0) ** m) * dfact)
        P[(m, m)] = pmm
        if m + 1 <= lmax:
            P[(m + 1, m)] = z * (2 * m + 1) * pmm
        for l in range(m + 2, lmax + 1):
            P[(l, m)] = ((2 * l - 1) * z * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sh(lmax: int, dirs: torch.Tensor) -> torch.Tensor:
    """(N, 3) unit directions -> (N, (lmax+1)^2) real SH values, ordered l-major, m=-l..l."""
    x, y, z = dirs[..., 0], dirs[..., 1], dirs[..., 2]
    P = _legendre_reduced(lmax, z)
    # c_m + i s_m = (x + i y)^m
    cs = [(torch.ones_like(x), torch.zeros_like(x))]
    for m in range(1, lmax + 1):
        c, s = cs[-1]
        cs.append((x * c - y * s, x * s + y * c))
    out = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            if m == 0:
                out.append(K * P[(l, 0)])
            elif m > 0:
                out.append(math.sqrt(2.0) * K * P[(l, am)] * cs[am][0])
            else:
                out.append(math.sqrt(2.0) * K * P[(l, am)] * cs[am][1])
    return torch.stack(out, -1)
