"""Adam on Gaussian parameters and on se(3) pose increments, float64 (oracle).

The paper refines splats and poses jointly by gradient descent on the multimodal loss
(Sec. III-C, final paragraph) without naming the optimiser; the refinement workload uses
Adam, with se(3) tangent updates for the poses:
    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2
    step = lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
    Gaussians: p <- p - step
    pose b:    delta = -step (6-vector, rho first);  W_b <- Exp(delta) W_b
"""
from __future__ import annotations

import numpy as np

from .geometry import perturb_pose


def adam_update(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-15):
    """One Adam step at (1-based) step t; returns new (p, m, v) as float64 arrays."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def pose_update(R, t_vec, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-15):
    """Adam on the tangent increment of one pose, then the left retraction Exp(delta) W."""
    delta, m, v = adam_update(np.zeros(6), g, m, v, step, lr, b1, b2, eps)
    R2, t2 = perturb_pose(R, t_vec, delta)
    return R2, t2, m, v
