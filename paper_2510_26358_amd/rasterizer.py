"""Torch-facing binding of libagsplat: device buffers, streams and autograd plumbing.

Every step of the rasteriser runs in the library's HIP kernels; this module only packs
pointers and shapes, allocates caller-owned buffers as torch tensors and passes the
current HIP stream.  There is no CPU fallback: without the built library, or without a
GPU, calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _fwd_out(out):
    """ags_fwd_out for (rgb, depth, alpha[, depth variance])."""
    return L.FwdOut(out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
                    out[3].data_ptr() if len(out) > 3 else None)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _i32(xs):
    return (C.c_int32 * len(xs))(*[int(x) for x in xs])


def _i64(xs):
    return (C.c_int64 * len(xs))(*[int(x) for x in xs])


class ViewSpec:
    """Static shape of a batch of views: sizes and each view's Gaussian range."""

    def __init__(self, widths, heights, g_begin, g_end):
        self.widths = [int(w) for w in widths]
        self.heights = [int(h) for h in heights]
        self.g_begin = [int(g) for g in g_begin]
        self.g_end = [int(g) for g in g_end]
        self._arr = (_i32(self.widths), _i32(self.heights), _i32(self.g_begin), _i32(self.g_end))
        self.c = L.Views(len(self.widths), *self._arr)

    @property
    def n_views(self):
        return len(self.widths)

    @property
    def pix_base(self):
        out = [0]
        for w, h in zip(self.widths, self.heights):
            out.append(out[-1] + w * h)
        return out

    @property
    def n_pixels(self):
        return self.pix_base[-1]

    def subset(self, b):
        return ViewSpec([self.widths[b]], [self.heights[b]], [self.g_begin[b]], [self.g_end[b]])

    @classmethod
    def from_scene(cls, scene):
        n = scene.n
        return cls([c.width for c in scene.cameras], [c.height for c in scene.cameras],
                   [c.g_begin for c in scene.cameras],
                   [c.g_end if c.g_end >= 0 else n for c in scene.cameras])


@dataclass
class SplatParams:
    """Gaussian parameters, structure-of-arrays float32 on the GPU."""
    means: torch.Tensor           # (3, N)
    log_scales: torch.Tensor      # (3, N)
    quats: torch.Tensor           # (4, N)
    opacity_logits: torch.Tensor  # (N,)
    sh: torch.Tensor              # (K, 3, N)
    sh_degree: int

    @property
    def n(self):
        return int(self.opacity_logits.shape[0])

    def tensors(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logits, self.sh]

    def c(self):
        return L.Gaussians(self.n, self.sh_degree, *[t.data_ptr() for t in self.tensors()])

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        return cls(f(scene.means.T), f(scene.log_scales.T), f(scene.quats.T),
                   f(scene.opacity_logits), f(np.transpose(scene.sh, (1, 2, 0))), scene.sh_degree)

    def zeros_like(self):
        return SplatParams(*[torch.zeros_like(t) for t in self.tensors()], self.sh_degree)

    @classmethod
    def empty(cls, n: int, sh_degree: int, device="cuda"):
        K = (sh_degree + 1) ** 2
        e = lambda *shape: torch.empty(*shape, device=device)
        return cls(e(3, n), e(3, n), e(4, n), e(n), e(K, 3, n), sh_degree)

    def narrow(self, k: int):
        """The first k Gaussians, as contiguous tensors."""
        return SplatParams(*[t[..., :k].contiguous() for t in self.tensors()], self.sh_degree)

    def clone(self):
        return SplatParams(*[t.clone() for t in self.tensors()], self.sh_degree)

    def to_numpy_aos(self):
        """(means (N,3), log_scales, quats, opacity_logits, sh (N,K,3)) as numpy."""
        return (self.means.T.cpu().numpy(), self.log_scales.T.cpu().numpy(),
                self.quats.T.cpu().numpy(), self.opacity_logits.cpu().numpy(),
                self.sh.permute(2, 0, 1).cpu().numpy())


def cameras_tensor(cameras, device="cuda"):
    """(B, 16) float32: R (row-major), t, fx, fy, cx, cy -- the ags_camera layout."""
    rows = []
    for c in cameras:
        rows.append(np.concatenate([np.asarray(c.R, np.float64).reshape(9), np.asarray(c.t, np.float64),
                                    [c.fx, c.fy, c.cx, c.cy]]))
    return torch.tensor(np.array(rows), dtype=torch.float32, device=device)


@dataclass
class LifecycleParams:
    """Thresholds of the lifecycle operations (see ags_lifecycle in include/agsplat.h)."""
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

    def c(self):
        return L.Lifecycle(int(self.do_prune), int(self.do_densify), int(self.do_reset), self.tau_opa, self.s_min,
                           self.s_max, self.grad_threshold, self.kappa, self.s_init, self.tau_reset,
                           self.split_scale)


@dataclass
class LossTargets:
    gt_rgb: torch.Tensor              # flat rgb layout
    mask: torch.Tensor | None         # (P,) uint8 or None
    l1_count: list
    depth_pix: torch.Tensor
    depth_val: torch.Tensor
    depth_sigma: torch.Tensor
    depth_offsets: list
    w_l1: float = 1.0
    lambda_lidar: float = 1.0
    ssim_weight: float = 0.0          # lambda of the D-SSIM part of L_3DGS (0: L1 only)
    sigma_mode: str = "fixed"         # LiDAR KL: "fixed" (sigma_u = sigma_L) or "rendered"
    sigma_floor: float = 1e-4         # m^2 added to the rendered depth variance

    @classmethod
    def from_scene(cls, scene, views: ViewSpec, device="cuda", masks=None, lidar=None, gt=None,
                   w_l1=1.0, lambda_lidar=1.0, ssim_weight=0.0, sigma_mode="fixed", sigma_floor=1e-4):
        gt = scene.gt_rgb if gt is None else gt
        lidar = scene.lidar if lidar is None else lidar
        flat = np.concatenate([np.asarray(g, np.float32).reshape(-1) for g in gt])
        mask_t, counts = None, [w * h for w, h in zip(views.widths, views.heights)]
        if masks is not None:
            mk = []
            counts = []
            for b, (w, h) in enumerate(zip(views.widths, views.heights)):
                m = np.zeros(w * h, np.uint8)
                if masks[b] is None:
                    m[:] = 1
                else:
                    m[np.asarray(masks[b], np.int64)] = 1
                counts.append(int(m.sum()))
                mk.append(m)
            mask_t = torch.from_numpy(np.concatenate(mk)).to(device)
        for b, d in enumerate(lidar or []):
            pb = np.asarray(d["pix"], np.int64)
            if b >= views.n_views and len(pb):
                raise ValueError(f"LiDAR targets given for view {b}, but there are {views.n_views} views")
            if len(pb) and (pb.min() < 0 or pb.max() >= views.widths[b] * views.heights[b]):
                raise ValueError(f"view {b}: LiDAR target pixel outside the {views.widths[b]}x{views.heights[b]} "
                                 f"image")
        pix = np.concatenate([np.asarray(d["pix"], np.int32) for d in lidar]) if lidar else np.zeros(0, np.int32)
        val = np.concatenate([np.asarray(d["depth"], np.float32) for d in lidar]) if lidar else np.zeros(0, np.float32)
        sig = np.concatenate([np.asarray(d["sigma"], np.float32) for d in lidar]) if lidar else np.zeros(0, np.float32)
        offs = [0]
        for d in (lidar or []):
            offs.append(offs[-1] + len(d["pix"]))
        while len(offs) < views.n_views + 1:
            offs.append(offs[-1])
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return cls(dev(flat), mask_t, counts, dev(pix), dev(val), dev(sig), offs, w_l1, lambda_lidar, ssim_weight,
                   sigma_mode, sigma_floor)

    def c(self):
        self._keep = (_i64(self.l1_count), _i64(self.depth_offsets))
        return L.Loss(self.gt_rgb.data_ptr(), self.mask.data_ptr() if self.mask is not None else None,
                      self._keep[0], self.depth_pix.data_ptr() if self.depth_pix.numel() else None,
                      self.depth_val.data_ptr() if self.depth_val.numel() else None,
                      self.depth_sigma.data_ptr() if self.depth_sigma.numel() else None,
                      self._keep[1], float(self.w_l1), float(self.lambda_lidar),
                      L.SIGMA_RENDERED if self.sigma_mode == "rendered" else L.SIGMA_FIXED,
                      float(self.sigma_floor), float(self.ssim_weight))


class Buffers:
    """Caller-owned device buffers for one batch shape and intersection capacity."""

    def __init__(self, sizes: L.Sizes, capacity: int, device):
        self.sizes = sizes
        self.capacity = int(capacity)
        self.saved = torch.empty(sizes.saved_bytes, dtype=torch.uint8, device=device)
        self.fwd_ws = torch.empty(sizes.fwd_ws_bytes, dtype=torch.uint8, device=device)
        self.bwd_ws = torch.empty(sizes.bwd_ws_bytes, dtype=torch.uint8, device=device)

    def view(self, off, count, dtype):
        nbytes = count * torch.tensor([], dtype=dtype).element_size()
        return self.saved[off:off + nbytes].view(dtype)

    def counters(self):
        """(K, V, overflow, K kept) -- synchronises."""
        return self.view(self.sizes.off_counters, 4, torch.int32).cpu().numpy().astype(np.int64)

    def n_listed(self) -> int:
        """Intersections in the per-tile lists (candidates the ellipse test keeps) -- synchronises."""
        return int(self.view(self.sizes.off_counters, 5, torch.int32)[4].item())


class Rasterizer:
    """A library context plus settings.  One instance per stream at a time."""

    def __init__(self, device: int = 0, tile: int = 16, batch: int = 256, px_per_thread: int = 1,
                 batch_bwd: int = 0, px_per_thread_bwd: int = 0, **settings):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libagsplat needs a ROCm GPU; none is visible")
        self.device = torch.device("cuda", device)
        cfg = L.Config()
        self.lib.ags_config_default(C.byref(cfg))
        cfg.tile, cfg.batch, cfg.px_per_thread = tile, batch, px_per_thread
        cfg.batch_bwd, cfg.px_per_thread_bwd = batch_bwd, px_per_thread_bwd
        for k, v in settings.items():
            if k == "bg":
                cfg.bg = (C.c_float * 3)(*v)
            else:
                setattr(cfg, k, v)
        self.cfg = cfg
        ctx = C.c_void_p()
        L.check(self.lib.ags_ctx_create(C.byref(ctx), device, C.byref(cfg)), "ags_ctx_create")
        self.ctx = ctx

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.ags_ctx_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def set_config(self, **kw):
        for k, v in kw.items():
            setattr(self.cfg, k, v)
        L.check(self.lib.ags_ctx_set_config(self.ctx, C.byref(self.cfg)), "ags_ctx_set_config")

    # ------------------------------------------------------------------ buffers
    def sizes(self, views: ViewSpec, n: int, sh_degree: int, capacity: int) -> L.Sizes:
        s = L.Sizes()
        L.check(self.lib.ags_buffer_sizes(C.byref(self.cfg), C.byref(views.c), n, sh_degree,
                                          int(capacity), C.byref(s)), "ags_buffer_sizes")
        return s

    def buffers(self, views: ViewSpec, n: int, sh_degree: int, capacity: int) -> Buffers:
        return Buffers(self.sizes(views, n, sh_degree, capacity), capacity, self.device)

    def outputs(self, views: ViewSpec, depth_var: bool = False):
        """(rgb, depth, alpha) buffers, plus the rendered depth variance when `depth_var`
        (needed by the rendered-variance LiDAR term)."""
        P = views.n_pixels
        out = (torch.empty(3 * P, device=self.device), torch.empty(P, device=self.device),
               torch.empty(P, device=self.device))
        return out + (torch.empty(P, device=self.device),) if depth_var else out

    # ------------------------------------------------------------------ calls
    def forward_into(self, params: SplatParams, cams: torch.Tensor, views: ViewSpec, buf: Buffers,
                     out):
        fo = _fwd_out(out)
        g = params.c()
        rc = self.lib.ags_render_fwd(self.ctx, C.byref(views.c), C.byref(g), _ptr(cams),
                                     buf.capacity, C.byref(fo), _ptr(buf.saved), _ptr(buf.fwd_ws),
                                     buf.sizes.fwd_ws_bytes, _stream())
        L.check(rc, "ags_render_fwd", self.ctx)

    def backward_into(self, params: SplatParams, cams, views: ViewSpec, buf: Buffers, out, grads,
                      pose_grad, upstream=None, loss: LossTargets | None = None, loss_out=None,
                      accumulate=False, stats=None, adam=None):
        """stats: optional (grad, count) float tensors [N] accumulating the densification
        statistic (|dL/d(u, v)| and the number of views seeing each Gaussian).
        adam: optional (hp: _lib.Adam, m: SplatParams, v: SplatParams, step: int32 tensor [1]):
        apply Adam to `params` in the same pass (ags_render_bwd_adam; grads.sh is then left
        unwritten)."""
        fo = _fwd_out(out)
        g = params.c()
        st = (None, None) if stats is None else (stats[0].data_ptr(), stats[1].data_ptr())
        gr = L.Grads(*[t.data_ptr() for t in grads.tensors()], pose_grad.data_ptr(), int(accumulate), *st)
        up = None
        lc = None
        if upstream is not None:
            d_rgb, d_depth, d_alpha = upstream
            up = L.Upstream(d_rgb.data_ptr() if d_rgb is not None else None,
                            d_depth.data_ptr() if d_depth is not None else None,
                            d_alpha.data_ptr() if d_alpha is not None else None)
        if loss is not None:
            lc = loss.c()
        if adam is not None:
            hp, m, v, step = adam
            mc, vc = m.c(), v.c()
            rc = self.lib.ags_render_bwd_adam(self.ctx, C.byref(views.c), C.byref(g), _ptr(cams), buf.capacity,
                                              C.byref(fo), _ptr(buf.saved), C.byref(up) if up is not None else None,
                                              C.byref(lc) if lc is not None else None, C.byref(gr),
                                              _ptr(loss_out), C.byref(hp), C.byref(mc), C.byref(vc), _ptr(step),
                                              _ptr(buf.bwd_ws), buf.sizes.bwd_ws_bytes, _stream())
            L.check(rc, "ags_render_bwd_adam", self.ctx)
            return
        rc = self.lib.ags_render_bwd(self.ctx, C.byref(views.c), C.byref(g), _ptr(cams), buf.capacity,
                                     C.byref(fo), _ptr(buf.saved), C.byref(up) if up is not None else None,
                                     C.byref(lc) if lc is not None else None, C.byref(gr),
                                     _ptr(loss_out), _ptr(buf.bwd_ws), buf.sizes.bwd_ws_bytes, _stream())
        L.check(rc, "ags_render_bwd", self.ctx)

    def check_finite(self, params: SplatParams) -> int:
        """Number of non-finite parameter values (debug aid; synchronises)."""
        bad = torch.zeros(1, dtype=torch.int32, device=self.device)
        g = params.c()
        L.check(self.lib.ags_check_finite(self.ctx, C.byref(g), _ptr(bad), _stream()), "ags_check_finite", self.ctx)
        return int(bad.item())

    def lifecycle_workspace(self, n: int) -> int:
        nbytes = C.c_size_t()
        L.check(self.lib.ags_lifecycle_workspace(n, C.byref(nbytes)), "ags_lifecycle_workspace")
        return int(nbytes.value)

    def lifecycle_into(self, params: SplatParams, m: SplatParams, v: SplatParams, lp: "LifecycleParams",
                       outs, n_out: torch.Tensor, actions: torch.Tensor | None, ws: torch.Tensor,
                       stats=None, noise=None):
        """One lifecycle pass into preallocated outputs (outs: three SplatParams of capacity
        >= 2 N; n_out: int32 [1]; ws: lifecycle_workspace(N) bytes).  No allocation, no sync."""
        gi, mi, vi = params.c(), m.c(), v.c()
        go, mo, vo = [o.c() for o in outs]
        sg = stats[0].data_ptr() if stats is not None else None
        sc = stats[1].data_ptr() if stats is not None else None
        lc = lp.c()
        rc = self.lib.ags_lifecycle_step(self.ctx, C.byref(lc), C.byref(gi), C.byref(mi), C.byref(vi), sg, sc,
                                         noise.data_ptr() if noise is not None else None, C.byref(go),
                                         C.byref(mo), C.byref(vo), _ptr(n_out),
                                         _ptr(actions) if actions is not None else None, _ptr(ws), ws.numel(),
                                         _stream())
        L.check(rc, "ags_lifecycle_step", self.ctx)

    def lifecycle(self, params: SplatParams, m: SplatParams, v: SplatParams, lp: "LifecycleParams",
                  stats=None, noise=None, capacity: int | None = None):
        """Prune / densify / reset (Sec. III-B lifecycle).  Returns (params, m, v, actions) with
        the new count; the outputs are fresh tensors (capacity 2 N, trimmed after one host
        read of the new count)."""
        n = params.n
        cap = capacity or max(2 * n, 1)
        outs = [SplatParams.empty(cap, params.sh_degree, self.device) for _ in range(3)]
        n_out = torch.zeros(1, dtype=torch.int32, device=self.device)
        actions = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        ws = torch.empty(max(self.lifecycle_workspace(n), 1), dtype=torch.uint8, device=self.device)
        self.lifecycle_into(params, m, v, lp, outs, n_out, actions, ws, stats=stats, noise=noise)
        k = int(n_out.item())
        return tuple(o.narrow(k) for o in outs) + (actions[:n],)

    def bin_records(self, views: ViewSpec, n: int, records: torch.Tensor, valid: torch.Tensor,
                    buf: Buffers):
        rc = self.lib.ags_bin_records(self.ctx, C.byref(views.c), n, _ptr(records), _ptr(valid),
                                      buf.capacity, _ptr(buf.saved), _ptr(buf.fwd_ws),
                                      buf.sizes.fwd_ws_bytes, _stream())
        L.check(rc, "ags_bin_records", self.ctx)

    def render(self, params: SplatParams, cams, views: ViewSpec, capacity: int | None = None,
               buf: Buffers | None = None, depth_var: bool = False):
        """Forward with automatic capacity growth (synchronises to read the counters).
        Returns (out, buffers)."""
        cap = capacity or (buf.capacity if buf is not None else max(1 << 16, 8 * views.n_pixels // 16))
        while True:
            if buf is None or buf.capacity < cap:
                buf = self.buffers(views, params.n, params.sh_degree, cap)
            out = self.outputs(views, depth_var)
            self.forward_into(params, cams, views, buf, out)
            k, v, over, keff = buf.counters()
            if not over:
                return out, buf
            cap = int(k * 1.25) + 1024

    # ------------------------------------------------------------------ tools
    def profile(self, enable=True):
        L.check(self.lib.ags_profile_enable(self.ctx, int(enable)), "ags_profile_enable")

    def profile_read(self):
        n = 32
        names = (C.c_char_p * n)()
        tot = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        nout = C.c_int()
        L.check(self.lib.ags_profile_read(self.ctx, n, names, tot, cnt, C.byref(nout)), "ags_profile_read")
        return {names[k].decode(): (tot[k], cnt[k]) for k in range(nout.value)}

    def profile_reset(self):
        L.check(self.lib.ags_profile_reset(self.ctx), "ags_profile_reset")


def split_views(flat_rgb, flat_depth, flat_alpha, views: ViewSpec):
    """Per-view (3,H,W), (H,W), (H,W) views of the flat output buffers."""
    out = []
    pb = views.pix_base
    for b, (w, h) in enumerate(zip(views.widths, views.heights)):
        out.append((flat_rgb[3 * pb[b]:3 * pb[b + 1]].view(3, h, w), flat_depth[pb[b]:pb[b + 1]].view(h, w),
                    flat_alpha[pb[b]:pb[b + 1]].view(h, w)))
    return out
