"""Gaussian-splat lifecycle operations (oracle; tests only): pruning, gradient-driven
densification (split / duplicate) and opacity reset, Sec. III-B "Gaussian Splats Lifecycle
Operations".

The paper fixes tau_opa = 0.01 and the size bounds 5e-5 < s < 0.3 and leaves gamma_g, kappa,
s_init, tau_reset and the split rule unstated; the readings taken here:
  * size s_j = the largest of the three scales, exp(max log-scale);
  * densification statistic g_j = (sum over views seeing j of |dL/d(u, v)|, pixel units) /
    (number of those views), accumulated by the backward;
  * prune if o_j < tau_opa or s_j > s_max or s_j < s_min;
  * else, if g_j > gamma_g: split if s_j > kappa (two children at mu + R(q) diag(s) eps_k with
    the given standard-normal eps_k, log-scales reduced by ln(split_scale), the rest copied);
    duplicate if s_j <= 2 s_init (the original and an exact copy);
  * opacity reset: if tau_opa <= o_j < tau_reset and s_min < s_j < s_max, the logit becomes
    logit(tau_reset) (in every output of j);
  * outputs keep input order (children and copies right after their parent's slot); the
    optimiser moments of new Gaussians (copies, children) are zero, survivors keep theirs.
The decisions are taken in float32 (the precision the kernel takes them in), the values in
float64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

KEEP, PRUNE, CLONE, SPLIT = 0, 1, 2, 3


@dataclass
class LifecycleParams:
    do_prune: bool = True
    do_densify: bool = True
    do_reset: bool = False
    tau_opa: float = 0.01
    s_min: float = 5e-5
    s_max: float = 0.3
    grad_threshold: float = 0.02
    kappa: float = 0.01
    s_init: float = 0.005
    tau_reset: float = 0.05
    split_scale: float = 1.6


def _f32_opacity(logits):
    x = np.asarray(logits, np.float32)
    return np.float32(1) / (np.float32(1) + np.exp(-x))


def _f32_size(log_scales):
    return np.exp(np.asarray(log_scales, np.float32).max(axis=1))


def classify(log_scales, logits, grad_accum, count, lp: LifecycleParams):
    """Per-Gaussian action (KEEP / PRUNE / CLONE / SPLIT) and reset flag, decided in float32."""
    o = _f32_opacity(logits)
    s = _f32_size(log_scales)
    g = np.asarray(grad_accum, np.float32) / np.maximum(np.asarray(count, np.float32), np.float32(1))
    f = np.float32
    act = np.full(len(o), KEEP, np.int64)
    if lp.do_prune:
        act[(o < f(lp.tau_opa)) | (s > f(lp.s_max)) | (s < f(lp.s_min))] = PRUNE
    if lp.do_densify:
        hot = (act == KEEP) & (np.asarray(count) > 0) & (g > f(lp.grad_threshold))
        act[hot & (s > f(lp.kappa))] = SPLIT
        act[hot & ~(s > f(lp.kappa)) & (s <= f(2 * lp.s_init))] = CLONE
    reset = np.zeros(len(o), bool)
    if lp.do_reset:
        reset = (act != PRUNE) & (o >= f(lp.tau_opa)) & (o < f(lp.tau_reset)) & (s > f(lp.s_min)) & (s < f(lp.s_max))
    return act, reset


def quat_rotation(q):
    """Rows of the rotation matrix of the normalised quaternion (w, x, y, z), float64."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def apply(params: dict, m: dict, v: dict, grad_accum, count, noise, lp: LifecycleParams):
    """params / m / v: dicts of per-Gaussian arrays (means (N,3), log_scales (N,3), quats (N,4),
    opacity_logits (N,), sh (N,K,3)); noise (N, 2, 3) standard normals for split children.
    Returns (new params, new m, new v, actions)."""
    act, reset = classify(params["log_scales"], params["opacity_logits"], grad_accum, count, lp)
    n = len(act)
    reset_logit = float(np.log(lp.tau_reset / (1.0 - lp.tau_reset)))
    rows, kinds = [], []          # (source index, 0 = copy with moments, 1 = new copy, 2/3 = child 0/1)
    for i in range(n):
        if act[i] == PRUNE:
            continue
        if act[i] == SPLIT:
            rows += [i, i]
            kinds += [2, 3]
        elif act[i] == CLONE:
            rows += [i, i]
            kinds += [0, 1]
        else:
            rows.append(i)
            kinds.append(0)
    rows = np.asarray(rows, np.int64)
    kinds = np.asarray(kinds, np.int64)
    out = {k: np.asarray(a, np.float64)[rows].copy() for k, a in params.items()}
    om = {k: np.asarray(a, np.float64)[rows].copy() for k, a in m.items()}
    ov = {k: np.asarray(a, np.float64)[rows].copy() for k, a in v.items()}
    new = kinds != 0
    for d in (om, ov):
        for k in d:
            d[k][new] = 0.0
    child = kinds >= 2
    if child.any():
        src = rows[child]
        R = quat_rotation(np.asarray(params["quats"], np.float64)[src])
        sc = np.exp(np.asarray(params["log_scales"], np.float64)[src])
        eps = np.asarray(noise, np.float64)[src, kinds[child] - 2]
        out["means"][child] = np.asarray(params["means"], np.float64)[src] + np.einsum("nij,nj->ni", R, sc * eps)
        out["log_scales"][child] = np.asarray(params["log_scales"], np.float64)[src] - np.log(lp.split_scale)
    out["opacity_logits"][reset[rows]] = reset_logit
    return out, om, ov, act
