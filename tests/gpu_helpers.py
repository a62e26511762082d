"""Drive the HIP path through the C ABI for a scene and return numpy results (tests only).

Nothing here computes any part of the rasteriser: it marshals inputs, calls the library
and converts outputs.  Comparisons against the oracle live in the tests themselves.
"""
from __future__ import annotations

import numpy as np
import torch

from paper_2510_26358_amd.rasterizer import (LossTargets, Rasterizer, SplatParams, ViewSpec,
                                             cameras_tensor, split_views)

# Tolerances stated for this path: colour and alpha 1e-4 absolute, depth 1e-4 * max(1, D),
# gradients 1e-3 relative.
TOL_RGB = 1e-4
TOL_ALPHA = 1e-4
TOL_DEPTH_REL = 1e-4
TOL_GRAD = 1e-3


def run_forward(scene, ras: Rasterizer, capacity=None, depth_var=False):
    views = ViewSpec.from_scene(scene)
    p = SplatParams.from_scene(scene)
    cams = cameras_tensor(scene.cameras)
    out, buf = ras.render(p, cams, views, capacity=capacity, depth_var=depth_var)
    torch.cuda.synchronize()
    res = []
    for b, (rgb, d, a) in enumerate(split_views(*out[:3], views)):
        res.append({"rgb": rgb.cpu().numpy(), "depth": d.cpu().numpy(), "alpha": a.cpu().numpy()})
    if depth_var:
        pb = views.pix_base
        for b in range(views.n_views):
            res[b]["depth_var"] = out[3][pb[b]:pb[b + 1]].cpu().numpy().reshape(views.heights[b], views.widths[b])
    return res, (p, cams, views, out, buf)


def saved_arrays(buf, views: ViewSpec):
    s = buf.sizes
    k, v, over, keff = buf.counters()
    t_final = buf.view(s.off_t_final, views.n_pixels, torch.float32).cpu().numpy()
    last = buf.view(s.off_last, views.n_pixels, torch.int32).cpu().numpy()
    recs = buf.view(s.off_records, s.n_pairs * 12, torch.float32).view(-1, 12).cpu().numpy()
    cnt = buf.view(s.off_pair_count, s.n_pairs, torch.int32).cpu().numpy()
    n_list = buf.n_listed()
    pairs = buf.view(s.off_tile_pairs, n_list, torch.int32).cpu().numpy().astype(np.int64)
    ranges = buf.view(s.off_ranges, 2 * s.n_tiles, torch.int32).view(-1, 2).cpu().numpy().astype(np.int64)
    keys = buf.fwd_ws[s.off_tile_keys:s.off_tile_keys + 4 * n_list].view(torch.int32).cpu().numpy()
    work = buf.view(s.off_work, s.n_work, torch.int32).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    return {"K": int(k), "V": int(v), "overflow": int(over), "K_kept": int(keff), "n_listed": n_list,
            "t_final": t_final,
            "last": last, "records": recs, "pair_count": cnt, "tile_pairs": pairs, "ranges": ranges,
            "tile_keys": keys.astype(np.int64) & 0xFFFFFFFF, "work": work}


def run_loss_backward(scene, ras: Rasterizer, masks=None, w_l1=1.0, lam=1.0, capacity=None, ssim_w=0.0,
                      gt=None, sigma_mode="fixed", sigma_floor=1e-4, stats=False):
    res, (p, cams, views, out, buf) = run_forward(scene, ras, capacity, depth_var=sigma_mode == "rendered")
    tg = LossTargets.from_scene(scene, views, masks=masks, w_l1=w_l1, lambda_lidar=lam, ssim_weight=ssim_w,
                                gt=gt, sigma_mode=sigma_mode, sigma_floor=sigma_floor)
    grads = p.zeros_like()
    pose = torch.zeros(views.n_views, 6, device="cuda")
    loss = torch.zeros(1, device="cuda")
    st = (torch.zeros(p.n, device="cuda"), torch.zeros(p.n, device="cuda")) if stats else None
    ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss, stats=st)
    torch.cuda.synchronize()
    g = grads.to_numpy_aos()
    names = ["means", "log_scales", "quats", "opacity_logits", "sh"]
    r = {"loss": float(loss.item()), "grads": dict(zip(names, g)), "pose": pose.cpu().numpy(),
         "fwd": res, "buf": buf, "views": views}
    if stats:
        r["stats"] = {"grad_accum": st[0].cpu().numpy(), "count": st[1].cpu().numpy()}
    return r


def grad_close(gpu, ref, exclude=None, rel=TOL_GRAD, frac=0.999):
    """Per-tensor norm check and per-element check on >= frac of the elements:
    ||d||_2 <= rel ||ref||_2 and |d_i| <= rel * max(|ref_i|, 1e-2 ||ref||_inf)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    if exclude is not None:
        keep = ~exclude
        gpu, ref = gpu[keep], ref[keep]
    d = gpu - ref
    nref = np.linalg.norm(ref)
    if nref == 0:
        return np.abs(d).max() <= 1e-12, "zero reference"
    ok_norm = np.linalg.norm(d) <= rel * nref
    bound = rel * np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max())
    good = np.abs(d) <= bound
    ok_elem = good.mean() >= frac
    return ok_norm and ok_elem, (f"norm rel {np.linalg.norm(d) / nref:.2e}, elem ok {good.mean():.5f}, "
                                 f"worst {np.abs(d / np.maximum(bound / rel, 1e-30)).max():.2e}")
