"""Joint map + pose refinement loop with a HIP-graph-captured step.

One step = batched forward render, fused L1 + LiDAR-KL backward (Sec. III-C), Adam on the
Gaussian parameters and Adam on each camera's se(3) increment followed by the left
retraction W_b <- Exp(delta_b) W_b (the paper refines splats and poses jointly through the
multimodal loss, Sec. III-C).  Every buffer is allocated once; the library calls only
enqueue kernels (no allocation, no host synchronisation, no memset nodes), so the whole
step is captured once and replayed.  The step counter lives in device memory.

The intersection count is data dependent: the capacity is fixed when capturing (with
headroom), and `check_capacity()` (one host read) reports an overflow so the caller can
re-capture with a larger capacity.  `save` / `load` checkpoint the loop's whole state
(parameters, Adam moments, poses, pose optimiser state, step counter) as an .npz file.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .rasterizer import LossTargets, Rasterizer, SplatParams, ViewSpec

FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")

DEFAULT_LR = {"means": 1e-3, "log_scales": 5e-3, "quats": 1e-3, "opacity": 5e-2, "sh0": 2.5e-3,
              "shrest": 1.25e-4, "pose": 1e-3}


class Refiner:
    def __init__(self, ras: Rasterizer, params: SplatParams, cams: torch.Tensor, views: ViewSpec,
                 targets: LossTargets, lr: dict | None = None, capacity: int | None = None,
                 headroom: float = 1.3, betas=(0.9, 0.999), eps=1e-15, fused_adam: bool = True):
        self.ras, self.p, self.cams, self.views, self.targets = ras, params, cams, views, targets
        self.fused_adam = fused_adam
        lr = {**DEFAULT_LR, **(lr or {})}
        self.hp = L.Adam(lr["means"], lr["log_scales"], lr["quats"], lr["opacity"], lr["sh0"], lr["shrest"],
                         lr["pose"], betas[0], betas[1], eps)
        dev = params.means.device
        if capacity is None:
            _, b = ras.render(params, cams, views)
            capacity = int(b.counters()[0] * headroom) + 4096
            del b
        self.buf = ras.buffers(views, params.n, params.sh_degree, capacity)
        self.out = ras.outputs(views, depth_var=targets.sigma_mode == "rendered")
        self.grads = params.zeros_like()
        self.m = params.zeros_like()
        self.v = params.zeros_like()
        B = views.n_views
        self.pose_grad = torch.zeros(B, 6, device=dev)
        self.pose_m = torch.zeros(B, 6, device=dev)
        self.pose_v = torch.zeros(B, 6, device=dev)
        self.step_no = torch.ones(1, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(1, device=dev)
        self.graph = None
        self._keep = None

    # ---------------------------------------------------------------- one step
    def step(self):
        """Enqueue one optimisation step on the current stream (no host sync)."""
        ras, lib = self.ras, self.ras.lib
        ras.forward_into(self.p, self.cams, self.views, self.buf, self.out)
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        if self.fused_adam:
            # backward and Adam in one pass over the Gaussians (the SH gradient stays in registers)
            ras.backward_into(self.p, self.cams, self.views, self.buf, self.out, self.grads, self.pose_grad,
                              loss=self.targets, loss_out=self.loss, adam=(self.hp, self.m, self.v, self.step_no))
        else:
            ras.backward_into(self.p, self.cams, self.views, self.buf, self.out, self.grads, self.pose_grad,
                              loss=self.targets, loss_out=self.loss)
            gr = L.Grads(*[t.data_ptr() for t in self.grads.tensors()], self.pose_grad.data_ptr(), 0)
            pc, mc, vc = self.p.c(), self.m.c(), self.v.c()
            L.check(lib.ags_adam_step(ras.ctx, C.byref(self.hp), C.byref(pc), C.byref(gr), C.byref(mc),
                                      C.byref(vc), C.c_void_p(self.step_no.data_ptr()), stream), "ags_adam_step",
                    ras.ctx)
        L.check(lib.ags_pose_step(ras.ctx, C.byref(self.hp), C.c_void_p(self.cams.data_ptr()), self.views.n_views,
                                  C.c_void_p(self.pose_grad.data_ptr()), C.c_void_p(self.pose_m.data_ptr()),
                                  C.c_void_p(self.pose_v.data_ptr()), C.c_void_p(self.step_no.data_ptr()), 1,
                                  stream), "ags_pose_step", ras.ctx)

    def capture(self, warmup: int = 0):
        """Capture one step into a HIP graph (after `warmup` eager steps)."""
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g
        return g

    def replay(self, n: int = 1):
        for _ in range(n):
            self.graph.replay()

    # ---------------------------------------------------------------- checkpoint / resume
    def state(self) -> dict:
        """Everything the loop carries between steps, as host numpy arrays: the parameters,
        both Adam moments, the camera array (poses), the pose optimiser state and the step."""
        torch.cuda.synchronize()
        out = {"sh_degree": np.int64(self.p.sh_degree), "cams": self.cams.cpu().numpy(),
               "pose_m": self.pose_m.cpu().numpy(), "pose_v": self.pose_v.cpu().numpy(),
               "step": self.step_no.cpu().numpy()}
        for tag, sp in (("p", self.p), ("m", self.m), ("v", self.v)):
            for name, t in zip(FIELDS, sp.tensors()):
                out[f"{tag}_{name}"] = t.cpu().numpy()
        return out

    def save(self, path: str):
        """Checkpoint to an .npz file (plain arrays, no pickled objects)."""
        np.savez(path, **self.state())

    def load(self, path: str):
        """Resume from a checkpoint written by `save` for the same Gaussian count and views:
        values are copied into the existing buffers, so a captured graph stays valid."""
        with np.load(path, allow_pickle=False) as z:
            if int(z["sh_degree"]) != self.p.sh_degree or z["p_means"].shape != tuple(self.p.means.shape) \
                    or z["cams"].shape != tuple(self.cams.shape):
                raise ValueError(f"{path}: checkpoint shape does not match this refiner")
            for tag, sp in (("p", self.p), ("m", self.m), ("v", self.v)):
                for name, t in zip(FIELDS, sp.tensors()):
                    t.copy_(torch.from_numpy(z[f"{tag}_{name}"]))
            self.cams.copy_(torch.from_numpy(z["cams"]))
            self.pose_m.copy_(torch.from_numpy(z["pose_m"]))
            self.pose_v.copy_(torch.from_numpy(z["pose_v"]))
            self.step_no.copy_(torch.from_numpy(z["step"]))
        torch.cuda.synchronize()

    def check_capacity(self) -> bool:
        """True when the last forward fitted its intersection capacity (synchronises)."""
        k, v, over, keff = self.buf.counters()
        return not over
