"""torch.autograd.Function wrappers around the library's forward and backward calls.

`render(...)` returns per-pixel colour, expected depth and alpha and back-propagates any
upstream gradient through `ags_render_bwd` (upstream mode).  `render_loss(...)` evaluates
the fused L1 + LiDAR-KL loss of Sec. III-C in the backward kernels and returns it as a
scalar whose backward scales the already computed gradients.  In both, the camera poses
receive a gradient through a zero "pose_delta" input (B, 6): the derivative with respect to
a left perturbation W_b <- Exp(delta_b) W_b, delta = (rho, phi).  That input is the point at
which the pose gradient is taken and must hold zeros: a non-zero value raises ValueError
instead of silently rendering at delta = 0 (move a camera by updating `cams`, e.g. with the
library's pose step).
"""
from __future__ import annotations

import torch

from .rasterizer import LossTargets, Rasterizer, SplatParams, ViewSpec


class _State:
    def __init__(self, ras: Rasterizer, cams, views: ViewSpec, sh_degree: int, capacity=None):
        self.ras, self.cams, self.views, self.sh_degree = ras, cams, views, sh_degree
        self.capacity = capacity
        self.buf = None


def _check_pose_delta(nonzero):
    """Raise if the pose input held a non-zero entry (`nonzero`: a device count taken before
    the render, read after the render's own synchronisation)."""
    if int(nonzero.item()) != 0:
        raise ValueError("pose_delta must be zero: it marks where the pose gradient is taken; "
                         "update the cameras to move them")


def _params(means, log_scales, quats, logits, sh, deg):
    return SplatParams(means.detach().contiguous(), log_scales.detach().contiguous(),
                       quats.detach().contiguous(), logits.detach().contiguous(),
                       sh.detach().contiguous(), deg)


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, logits, sh, pose_delta, st: _State):
        nonzero = torch.count_nonzero(pose_delta.detach())
        p = _params(means, log_scales, quats, logits, sh, st.sh_degree)
        out, buf = st.ras.render(p, st.cams, st.views, capacity=st.capacity, buf=st.buf)
        _check_pose_delta(nonzero)
        st.buf = buf
        st.capacity = buf.capacity
        ctx.st = st
        ctx.p = p
        ctx.out = out
        ctx.buf = buf
        return out

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha):
        st, p = ctx.st, ctx.p
        grads = p.zeros_like()
        pose = torch.zeros(st.views.n_views, 6, device=p.means.device)
        up = tuple(g.contiguous() if g is not None else None for g in (g_rgb, g_depth, g_alpha))
        st.ras.backward_into(p, st.cams, st.views, ctx.buf, ctx.out, grads, pose, upstream=up)
        return (*grads.tensors(), pose, None)


def render(means, log_scales, quats, opacity_logits, sh, pose_delta, ras: Rasterizer, cams,
           views: ViewSpec, sh_degree: int, capacity=None):
    """Differentiable batched render of all views: returns flat (rgb, depth, alpha)."""
    st = _State(ras, cams, views, sh_degree, capacity)
    return _RenderFn.apply(means, log_scales, quats, opacity_logits, sh, pose_delta, st)


class _RenderLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, logits, sh, pose_delta, st: _State,
                targets: LossTargets):
        nonzero = torch.count_nonzero(pose_delta.detach())
        p = _params(means, log_scales, quats, logits, sh, st.sh_degree)
        out, buf = st.ras.render(p, st.cams, st.views, capacity=st.capacity, buf=st.buf)
        _check_pose_delta(nonzero)
        st.buf = buf
        grads = p.zeros_like()
        pose = torch.zeros(st.views.n_views, 6, device=p.means.device)
        loss = torch.zeros(1, device=p.means.device)
        st.ras.backward_into(p, st.cams, st.views, buf, out, grads, pose, loss=targets, loss_out=loss)
        ctx.grads = (*grads.tensors(), pose)
        ctx.outputs = out
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        return (*[t * g for t in ctx.grads], None, None)


def render_loss(means, log_scales, quats, opacity_logits, sh, pose_delta, ras: Rasterizer, cams,
                views: ViewSpec, sh_degree: int, targets: LossTargets, capacity=None):
    """Fused L1 + LiDAR-KL loss of the batched render (scalar, differentiable)."""
    st = _State(ras, cams, views, sh_degree, capacity)
    return _RenderLossFn.apply(means, log_scales, quats, opacity_logits, sh, pose_delta, st, targets)
