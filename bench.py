"""Benchmark: forward + backward Mpixel/s of the batched multi-view rasteriser vs a per-view
loop of the same kernels, with the L1 + LiDAR-KL loss, on one MI355X.

Workload (default): 1M orchard-row Gaussians (SH degree 3) seen by a 4-camera rig
(yaw 0, +60, -60, 180 deg) at 1280x800; target images are renders of the unperturbed map,
the rendered state has means jittered by 1 cm and poses perturbed; LiDAR depth targets on
~5 % of the pixels.  One step = projection, binning, depth/tile sorts, raster forward,
LiDAR adjoint, raster backward with the fused L1 prologue, projection/pose backward -- all
views in one launch per stage.  Inputs are resident in HBM before timing starts.

Prints one JSON line (rank 0).  `--gpus N` with N > 1 exits: the measurement is of one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpixel/s, batched multi-view vs per-view loop, at oracle tolerance"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X published vector FP32 peak (packed, 2-wide FP32 instructions)
# Attainable without packed FP32 (the library compiles all device code without it): a wave64
# FP32 instruction occupies a 16-lane SIMD for 4 cycles, so 256 CU x 4 SIMD x 16 lanes x
# 2 FLOP (FMA) x 2.4 GHz = 78.6 TFLOP/s; reported beside the published peak.
FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
TRIALS = 5  # timing: median over this many trials of `steps` replays each
# Algorithmic FLOP per (pixel, Gaussian) pair evaluated: forward ~20 + 1 exp,
# backward ~60 + 1 exp; the exp is counted as one FLOP.
FLOP_PER_PAIR = {"raster_fwd": 21, "raster_bwd": 61}
# Algorithmic FLOP of the D-SSIM term per pixel and colour channel (no halo recomputation):
# five window moments by two 11-tap passes (220), s and its three partial derivatives (~40),
# three 11-tap passes back (132), the final combination (~8).
SSIM_FLOP_PER_PIXEL_CHANNEL = 400
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2510_26358_amd import scenes
    if name == "multi_view":
        sc = scenes.multi_view_scene()
    elif name == "single_view":
        sc = scenes.single_view_scene()
    elif name == "refine":
        sc = scenes.refinement_scene()
    elif name == "submaps":
        sc = scenes.submap_scene()
    elif name == "tiny":
        sc = scenes.tiny_scene()
    else:
        raise SystemExit(f"unknown workload {name}")
    return sc


def setup(sc, ras):
    """Upload the perturbed state; targets = renders of the unperturbed map."""
    import torch
    from paper_2510_26358_amd import scenes
    from paper_2510_26358_amd.rasterizer import (LossTargets, SplatParams, ViewSpec, cameras_tensor)
    views = ViewSpec.from_scene(sc)
    p_gt = SplatParams.from_scene(sc)
    cams_gt = cameras_tensor(sc.cameras)
    out_gt, buf = ras.render(p_gt, cams_gt, views)
    torch.cuda.synchronize()
    gt = [out_gt[0][3 * a:3 * b].view(3, h, w).cpu().numpy() for a, b, w, h in
          zip(views.pix_base[:-1], views.pix_base[1:], views.widths, views.heights)]
    if sc.name != "tiny":
        st = scenes.perturb(sc, seed=77)
    else:
        st = sc
    p = SplatParams.from_scene(st)
    cams = cameras_tensor(st.cameras)
    tg = LossTargets.from_scene(sc, views, gt=gt if sc.name != "tiny" else None)
    del out_gt, buf
    return p, cams, views, tg


def calibrate(ras, p, cams, views, headroom=1.15):
    out, buf = ras.render(p, cams, views)
    k, v, over, keff = buf.counters()
    cap = int(k * headroom) + 4096
    return cap, int(k), int(v)


def time_steps(fn, steps, warmup):
    """Seconds per step of exactly `steps` steps after `warmup` untimed ones, bracketed by a
    device synchronisation on both sides (the headline timing)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def time_trials(fn, steps, trials=TRIALS):
    """The measurement rule of the throughput table: `trials` trials of `steps` replays, each
    bracketed by HIP events on the current stream; the median trial's ms per step, and every
    trial's (called after the warm-up of `time_steps`)."""
    import torch
    stream = torch.cuda.current_stream()
    per = []
    for _ in range(trials):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) / steps)
    return {"rule": f"median of {trials} trials x {steps} replays (HIP events)",
            "median_ms": round(float(np.median(per)), 4), "trials_ms": [round(x, 4) for x in per]}


def measure_lifecycle(ras, p, cams, views, buf, out, grads, pose, tg, loss, args, t_b):
    """The step with the densification statistic accumulated by the backward, then the
    lifecycle pass over all Gaussians with that statistic (paper thresholds), timed on its own
    (HIP events around the pass); the pass is HBM-bound: algorithmic bytes = the parameters and
    both Adam moments read once per input and written once per output, plus the statistic,
    the split noise of split parents and the action bytes."""
    import torch
    from paper_2510_26358_amd.rasterizer import LifecycleParams, SplatParams
    n, K = p.n, (p.sh_degree + 1) ** 2
    stats = (torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"))

    def step_st():
        ras.forward_into(p, cams, views, buf, out)
        ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss, stats=stats)

    timed = step_st
    if not args.no_graph:
        for _ in range(args.warmup):
            step_st()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step_st()
        timed = g.replay
    t_st = time_steps(timed, args.steps, args.warmup)
    log(f"[bench] step accumulating the densification statistic: {t_st * 1e3:.3f} ms/step "
        f"(+{(t_st - t_b) * 1e6:.1f} us)")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4242)
    m = SplatParams(*[torch.randn(t.shape, device="cuda", generator=gen) for t in p.tensors()], p.sh_degree)
    v = SplatParams(*[torch.rand(t.shape, device="cuda", generator=gen) for t in p.tensors()], p.sh_degree)
    noise = torch.randn(n, 2, 3, device="cuda", generator=gen)
    outs = [SplatParams.empty(2 * n, p.sh_degree) for _ in range(3)]
    n_out = torch.zeros(1, dtype=torch.int32, device="cuda")
    actions = torch.empty(n, dtype=torch.uint8, device="cuda")
    ws = torch.empty(ras.lifecycle_workspace(n), dtype=torch.uint8, device="cuda")
    lp = LifecycleParams(do_reset=True)

    def run():
        ras.lifecycle_into(p, m, v, lp, outs, n_out, actions, ws, stats=stats, noise=noise)

    for _ in range(args.warmup):
        run()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        run()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    k = int(n_out.item())
    hist = torch.bincount(actions.to(torch.int64), minlength=4).cpu().tolist()
    row_bytes = 4 * (11 + 3 * K)
    nbytes = 3 * row_bytes * (n + k) + 8 * n + n + 24 * hist[3]
    gbs = nbytes / (ms * 1e-3) / 1e9
    res = {"ms_per_step_with_statistic": round(t_st * 1e3, 4),
           "statistic_overhead_us": round((t_st - t_b) * 1e6, 1),
           "n_in": n, "n_out": k, "keep": hist[0], "prune": hist[1], "duplicate": hist[2], "split": hist[3],
           "pass_ms": round(ms, 4),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_pass": nbytes}}
    log(f"[bench] lifecycle pass over {n} Gaussians -> {k}: {ms:.4f} ms, {gbs:.0f} GB/s ({res})")
    del outs, m, v
    return res


def measure_voxel_map(ras, args, n_points=1 << 20, tau=1 << 20, warm_calls=8, timed_calls=6):
    """Voxel-map insertion calls along a synthetic row: each call brings 2^20 points uniform in
    a 6 x 3 x 3 m window (a camera rig's view of a canopy row, voxel 0.05 m) that advances
    1.5 m per call, so about a quarter of the voxels are new; the resident set is bounded by
    2^20 splats (SH degree 3).  The first calls fill the resident set; the timed ones run in
    the steady state (new splats in, as many least recently used out to the host store).
    Reported: wall time per call (host-synchronous: includes the reload copy over PCIe; the
    offloaded rows leave on the map's copy stream and reach the host store on a host thread
    after the call returns, which is timed apart by waiting for it before the next call),
    per-stage GPU times
    (HIP events), and the roofline of the dominant kernel, the resident-set rebuild (HBM:
    every listed row written, 3 x 4 x 59 B, and read from the previous set or the reload
    staging, 24 B of point and colour for a new one)."""
    import torch
    from paper_2510_26358_amd.voxel_map import VoxelMap
    gm = VoxelMap(ras, voxel=0.05, sh_degree=3, tau=tau, max_ids=1 << 23, max_points=n_points)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9090)
    scale = torch.tensor([6.0, 3.0, 3.0], device="cuda")
    row_bytes = 3 * 4 * gm.F

    def call(t):
        pts = torch.rand(n_points, 3, device="cuda", generator=gen) * scale
        pts[:, 0] += 1.5 * t
        pts[:, 1] -= 1.5
        cols = torch.rand(n_points, 3, device="cuda", generator=gen)
        torch.cuda.synchronize()
        n_in = gm.n
        w0 = time.perf_counter()
        _, c = gm.insert(pts, cols, t)
        wall = time.perf_counter() - w0
        f0 = time.perf_counter()
        gm.sync()
        flush = time.perf_counter() - f0
        listed = n_in + c["n_new"] + c["n_reloaded"]
        rebuild = row_bytes * (n_in + c["n_reloaded"] + listed) + 24 * c["n_new"]
        pcie = row_bytes * (c["n_reloaded"] + c["n_evicted"])
        return wall * 1e3, flush * 1e3, rebuild, pcie, c

    for t in range(warm_calls):
        call(t)
    ras.profile(True)
    ras.profile_reset()
    recs = [call(warm_calls + k) for k in range(timed_calls)]
    torch.cuda.synchronize()
    prof = ras.profile_read()
    ras.profile(False)
    stage = {k: round(v[0] / timed_calls, 4) for k, v in prof.items() if k.startswith("map_") and v[1] > 0}
    life = lifecycle_over_map(ras, gm, gen, warm_calls + timed_calls)
    mean = lambda k: sum(r[k] for r in recs) / len(recs)
    wall, flush, rebuild, pcie = mean(0), mean(1), mean(2), mean(3)
    reb_ms = stage.get("map_rebuild", float("nan"))
    gbs = rebuild / (reb_ms * 1e-3) / 1e9
    res = {"points_per_call": n_points, "tau": tau, "calls_timed": timed_calls,
           "ms_per_call_wall": round(wall, 4), "host_store_ms_after_return": round(flush, 4),
           "mpoints_per_s_wall": round(n_points / (wall * 1e-3) / 1e6, 2), "stage_ms_per_call": stage,
           "new_per_call": round(sum(r[4]["n_new"] for r in recs) / len(recs)),
           "evicted_per_call": round(sum(r[4]["n_evicted"] for r in recs) / len(recs)),
           "reloaded_per_call": round(sum(r[4]["n_reloaded"] for r in recs) / len(recs)),
           "n_ids": recs[-1][4]["n_ids"], "n_resident": recs[-1][4]["n_resident"],
           "pcie_bytes_per_call": round(pcie),
           "pcie_gbs": round(pcie / (stage.get("map_copy", float("nan")) * 1e-3) / 1e9, 2),
           "roofline": {"kernel": "map_rebuild_kernel", "bound": "hbm", "achieved": round(gbs, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "bytes_per_launch": round(rebuild)},
           "lifecycle_pass": life}
    log(f"[bench] voxel map: {wall:.3f} ms/call wall, {res}")
    gm.close()
    del gm
    torch.cuda.empty_cache()
    return res


def _source_digest(stage):
    import hashlib
    src = {"raster_bwd": "raster.hip", "raster_fwd": "raster.hip", "project_bwd": "project_bwd.hip",
           "project_fwd": "project.hip"}.get(stage)
    if src is None:
        return None
    h = hashlib.sha256()
    for f in (src, "common.h"):
        with open(os.path.join(ROOT, "paper_2510_26358_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(stage, workload, launch=None):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
    this kernel and workload (for the launch configuration `launch` = (tile, pixels per
    thread, LDS batch) when the summary lists several), or None when absent or when the
    kernel source changed since."""
    path = os.path.join(PROFILES, f"{stage}_{workload}_counters.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != _source_digest(stage):
        return None
    key = "hbm_bytes_per_launch"
    if launch is not None and f"{key}[{','.join(str(x) for x in launch)}]" in vals:
        key = f"{key}[{','.join(str(x) for x in launch)}]"
    elif launch is not None and any(k.startswith(key + "[") for k in vals):
        return None
    try:
        return int(float(vals[key]))
    except (KeyError, ValueError):
        return None


def dominant_roofline(prof, views, buf, sizes, n_steps, n_gauss, sh_k, workload, launch=None):
    """Roofline of the slowest stage, from the library's per-stage HIP events over a timed
    pass (events on the launch stream); the algorithmic work of one launch is the work unit (one
    (pixel, Gaussian) pair of the raster kernels) times its FLOP."""
    import torch
    stages = {k: v for k, v in prof.items() if v[1] > 0}
    name = max(stages, key=lambda k: stages[k][0])
    ms_avg = stages[name][0] / stages[name][1]
    P = views.n_pixels
    last = buf.view(sizes.off_last, P, torch.int32).cpu().numpy().astype(np.int64)
    evals = int(last.sum())
    k, v, over, keff = buf.counters()
    info = {"stage": name, "avg_ms": ms_avg, "pairs_evaluated": evals, "K": int(k), "V": int(v)}
    traffic = measured_traffic(name, workload, launch)
    if name in FLOP_PER_PAIR:
        achieved = evals * FLOP_PER_PAIR[name] / (ms_avg * 1e-3) / 1e12
        rf = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
              "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": traffic,
              "peak_nonpacked": round(FP32_NONPACKED_TFLOPS, 2),
              "frac_nonpacked": round(achieved / FP32_NONPACKED_TFLOPS, 4),
              "work": f"{evals} (pixel, Gaussian) pairs x {FLOP_PER_PAIR[name]} FLOP"}
    else:
        # HBM-bound stages: algorithmic bytes per launch
        F = 11 + 3 * sh_k
        Q = sizes.n_pairs
        if name == "project_bwd":
            by = 4 * F * n_gauss * 2 + 52 * int(v) + 4 * Q
        elif name == "project_fwd":
            # parameters once; per visible pair its 48-byte record and its 64-byte adjoint row
            # zeroed for the backward; per pair its tile count and depth key
            by = 4 * F * n_gauss + 48 * int(v) + 8 * Q + 64 * int(v)
        elif name == "adam":
            by = 7 * 4 * F * n_gauss
        else:
            by = 8 * Q + 84 * int(v) + 44 * int(keff)
        achieved = by / (ms_avg * 1e-3) / 1e9
        rf = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
              "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic}
    return rf, info


def stage_rooflines(stage_ms, evals, P, N, sh_k, Q, V, K, n_targets, step_ms, fused_adam=False):
    """Every stage against its bound from the per-stage HIP-event times: algorithmic bytes
    (HBM-bound stages) or FLOP (raster) per launch, from the sizes below; plus the whole
    step's algorithmic bytes over its time (the HBM fraction of the step).  With the fused
    backward + Adam the projection backward also carries Adam's bytes, less the SH gradient's
    write and re-read and the second read of the SH coefficients.  The backward's accumulators
    are zeroed in the forward (the adjoint rows by the projection, the dense depth adjoint by
    the raster forward); a separate clear stage runs only for a backward that cannot rely on
    that."""
    F = 11 + 3 * sh_k
    byts = {
        "project_fwd": 4 * F * N + 48 * V + 8 * Q + 64 * V,
        "binning": 8 * Q + 84 * V + 44 * K,
        "lidar_adjoint": 16 * n_targets,
        "project_bwd": 2 * 4 * F * N + 56 * V + 24 * N,
        "raster_fwd": 28 * P + 4 * P,
        "raster_bwd": 44 * P,
    }
    if stage_ms.get("clear", 0) > 0:
        byts["clear"] = 4 * Q + 64 * V + 4 * P
    if "adam" in stage_ms:
        byts["adam"] = 7 * 4 * F * N
    elif fused_adam:
        byts["project_bwd"] += 7 * 4 * F * N - 3 * 4 * 3 * sh_k * N
    out = {}
    for name, ms in stage_ms.items():
        if ms <= 0:
            continue
        if name in FLOP_PER_PAIR:
            a = evals * FLOP_PER_PAIR[name] / (ms * 1e-3) / 1e12
            out[name] = {"ms": ms, "bound": "alu", "achieved": round(a, 2), "unit": "TFLOP/s",
                         "frac": round(a / FP32_PEAK_TFLOPS, 3),
                         "frac_nonpacked": round(a / FP32_NONPACKED_TFLOPS, 3)}
        elif name in byts:
            a = byts[name] / (ms * 1e-3) / 1e9
            out[name] = {"ms": ms, "bound": "hbm", "achieved": round(a, 1), "unit": "GB/s",
                         "frac": round(a / HBM_PEAK_GBS, 3)}
    total = sum(byts.values())
    out["step"] = {"ms": round(step_ms, 4), "bound": "hbm", "algorithmic_bytes": int(total),
                   "achieved": round(total / (step_ms * 1e-3) / 1e9, 1), "unit": "GB/s",
                   "frac": round(total / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)}
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def sample_pixels(sc, px_per_view, seed):
    """Seeded pixel sample per view (sorted flat indices) and the scene restricted to it: the
    L1 mask is the sample and only the LiDAR targets inside it are kept."""
    rng = np.random.default_rng(seed)
    samples = [np.sort(rng.choice(c.width * c.height, min(px_per_view, c.width * c.height), replace=False))
               for c in sc.cameras]
    sub = sc.copy()
    sub.lidar = []
    for lid, pix in zip(sc.lidar, samples):
        keep = np.isin(lid["pix"], pix)
        sub.lidar.append({k: np.asarray(v)[keep] for k, v in lid.items()})
    return sub, samples


def gpu_masked_step(ras, sub, samples, lam):
    """The HIP path on the sampled objective in the rasteriser's current launch configuration:
    forward outputs at the sample, loss, every gradient and the poses (generator inputs only)."""
    import torch
    from paper_2510_26358_amd.rasterizer import LossTargets, SplatParams, ViewSpec, cameras_tensor
    views = ViewSpec.from_scene(sub)
    p = SplatParams.from_scene(sub)
    cams = cameras_tensor(sub.cameras)
    out, buf = ras.render(p, cams, views)
    tg = LossTargets.from_scene(sub, views, masks=samples, w_l1=1.0, lambda_lidar=lam)
    grads = p.zeros_like()
    pose = torch.zeros(views.n_views, 6, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss)
    torch.cuda.synchronize()
    pb = views.pix_base
    fwd = []
    for b, pix in enumerate(samples):
        rgb = out[0][3 * pb[b]:3 * pb[b + 1]].view(3, -1)[:, torch.from_numpy(pix).cuda()].T.cpu().numpy()
        fwd.append({"rgb": rgb, "depth": out[1][pb[b]:pb[b + 1]][torch.from_numpy(pix).cuda()].cpu().numpy(),
                    "alpha": out[2][pb[b]:pb[b + 1]][torch.from_numpy(pix).cuda()].cpu().numpy()})
    names = ["means", "log_scales", "quats", "opacity_logits", "sh"]
    res = {"loss": float(loss.item()), "grads": dict(zip(names, grads.to_numpy_aos())), "pose": pose.cpu().numpy(),
           "fwd": fwd}
    del out, buf, grads, p
    return res


def parity_report(gpu, ref, samples):
    """Element-wise comparison at the stated tolerances (colour / alpha 1e-4, depth
    1e-4 max(1, D), gradients 1e-3 relative per tensor, the same for the poses); pixels whose
    result hinges on a decision rounding could flip (flagged by the oracle) and the Gaussians
    they touch are set aside and counted."""
    worst = {"rgb": 0.0, "alpha": 0.0, "depth_rel": 0.0}
    n_amb = 0
    for g, r, pix in zip(gpu["fwd"], ref["views"], samples):
        idx = np.searchsorted(r["pix"], pix)
        ok = ~r["ambiguous"][idx]
        n_amb += int((~ok).sum())
        worst["rgb"] = max(worst["rgb"], float(np.abs(g["rgb"] - r["rgb"][idx])[ok].max(initial=0)))
        worst["alpha"] = max(worst["alpha"], float(np.abs(g["alpha"] - r["alpha"][idx])[ok].max(initial=0)))
        worst["depth_rel"] = max(worst["depth_rel"], float(
            (np.abs(g["depth"] - r["depth"][idx]) / np.maximum(1.0, np.abs(r["depth"][idx])))[ok].max(initial=0)))
    keep = ~ref["amb_gauss"]
    gn = {}
    for name, g in gpu["grads"].items():
        rr = np.asarray(ref["grads"][name], np.float64)[keep]
        d = np.asarray(g, np.float64)[keep] - rr
        gn[name] = float(np.linalg.norm(d) / max(np.linalg.norm(rr), 1e-30))
    pose_rel = float(np.linalg.norm(gpu["pose"] - ref["pose"]) / max(np.linalg.norm(ref["pose"]), 1e-30))
    loss_rel = abs(gpu["loss"] - ref["loss"]) / max(1.0, abs(ref["loss"]))
    n_px = int(sum(len(x) for x in samples))
    ok = (worst["rgb"] <= 1e-4 and worst["alpha"] <= 1e-4 and worst["depth_rel"] <= 1e-4 and loss_rel <= 1e-4
          and all(v <= 1e-3 for v in gn.values()) and pose_rel <= 1e-3 and n_amb <= 0.005 * n_px)
    return {"pass": bool(ok), "pixels": n_px, "ambiguous": n_amb,
            "excluded_gaussians": int(ref["amb_gauss"].sum()),
            "max_rgb": float(f"{worst['rgb']:.3g}"), "max_alpha": float(f"{worst['alpha']:.3g}"),
            "max_depth_rel": float(f"{worst['depth_rel']:.3g}"), "loss_rel": float(f"{loss_rel:.3g}"),
            "grad_norm_rel": {k: float(f"{v:.3g}") for k, v in gn.items()}, "pose_rel": float(f"{pose_rel:.3g}")}


def oracle_leg(sc, ras, px_per_view, seed=5, lam=1.0, single_thread_px=0):
    """Parity of the HIP path in its timed launch configuration against the FP64 oracle on a
    seeded pixel sample of every view, and the oracle's own time for that sample (all host
    threads), plus, if asked, the oracle on one thread over a smaller sample of view 0."""
    import torch
    from oracle.render import loss_and_grads
    from oracle.settings import RenderSettings
    sub, samples = sample_pixels(sc, px_per_view, seed)
    gpu = gpu_masked_step(ras, sub, samples, lam)
    threads = torch.get_num_threads()
    t0 = time.perf_counter()
    ref = loss_and_grads(sub, RenderSettings(), masks=samples, lam=lam)
    dt = time.perf_counter() - t0
    parity = parity_report(gpu, ref, samples)
    n_px = parity["pixels"]
    cpu = {"value": round(n_px / dt / 1e6, 8), "unit": "Mpixel/s", "cores": threads, "kind": "oracle",
           "sample": f"{n_px} seeded pixels over the {len(sc.cameras)} views (L1 on the sample, LiDAR targets "
                     f"inside it), fwd+bwd over all {sc.n} Gaussians, {dt:.1f} s",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if single_thread_px:
        one, samples1 = sample_pixels(sc, single_thread_px, seed + 1)
        one.cameras, one.lidar, one.gt_rgb = one.cameras[:1], one.lidar[:1], one.gt_rgb[:1]
        torch.set_num_threads(1)
        try:
            t1 = time.perf_counter()
            loss_and_grads(one, RenderSettings(), masks=samples1[:1], lam=lam)
            d1 = time.perf_counter() - t1
        finally:
            torch.set_num_threads(threads)
        cpu["single_thread"] = {"value": round(len(samples1[0]) / d1 / 1e6, 8), "cores": 1,
                                "sample": f"{len(samples1[0])} seeded pixels of view 0, {d1:.1f} s"}
    return parity, cpu


def oracle_time(sc, samples, threads, lam=1.0):
    """Seconds the FP64 oracle takes for fwd + bwd of the sampled objective on `threads`
    host threads (None: all of torch's)."""
    import torch
    from oracle.render import loss_and_grads
    from oracle.settings import RenderSettings
    before = torch.get_num_threads()
    if threads:
        torch.set_num_threads(threads)
    try:
        t0 = time.perf_counter()
        loss_and_grads(sc, RenderSettings(), masks=samples, lam=lam)
        return time.perf_counter() - t0
    finally:
        torch.set_num_threads(before)


def oracle_other_configs():
    """The oracle's time on the tiny configuration's full image (2,000 Gaussians, 12,288 px) and
    on seeded 16 x 16 tiles of the single-view configuration (300k Gaussians; 64 tiles, 16,384
    px, on all host threads, 16 of them on one thread), in Mpixel/s."""
    import torch
    from paper_2510_26358_amd import scenes
    out = {}
    tiny = scenes.tiny_scene()
    full = [np.arange(tiny.cameras[0].width * tiny.cameras[0].height)]
    sv = scenes.single_view_scene()
    cam = sv.cameras[0]
    rng = np.random.default_rng(7)
    T, ntx = 16, (cam.width + 15) // 16
    tiles = rng.choice(ntx * ((cam.height + 15) // 16), 64, replace=False)
    pix = []
    for t in tiles:
        ys, xs = np.mgrid[(t // ntx) * T:min(cam.height, (t // ntx) * T + T), (t % ntx) * T:min(cam.width, (t % ntx) * T + T)]
        pix.append((ys * cam.width + xs).ravel())
    samp64 = [np.unique(np.concatenate(pix))]
    samp16 = [np.unique(np.concatenate(pix[:16]))]
    keep = np.isin(sv.lidar[0]["pix"], samp64[0])
    sv.lidar = [{k: np.asarray(v)[keep] for k, v in sv.lidar[0].items()}]
    runs = (("tiny_full_image", tiny, full, full), ("single_view_tiles", sv, samp64, samp16))
    for name, sc, smp_all, smp_one in runs:
        rec = {"n_gaussians": sc.n}
        for label, th, smp in (("all_threads", None, smp_all), ("one_thread", 1, smp_one)):
            n_px = int(sum(len(x) for x in smp))
            if th == 1 and smp is not smp_all:
                lid = sc.lidar[0]
                sc = sc.copy()
                k1 = np.isin(lid["pix"], smp[0])
                sc.lidar = [{k: np.asarray(v)[k1] for k, v in lid.items()}]
            dt = oracle_time(sc, smp, th)
            rec[label] = {"value": round(n_px / dt / 1e6, 8), "unit": "Mpixel/s", "pixels": n_px,
                          "cores": th or torch.get_num_threads(), "seconds": round(dt, 2)}
        out[name] = rec
    return out


def lifecycle_over_map(ras, gm, gen, frame):
    """A lifecycle pass over the map's full resident set (ags_lifecycle_step, then
    ags_map_lifecycle: retirements, new ids keyed like their parents, the rows packed into the
    resident set), then the next insertion call, which offloads the rows above tau.  The
    densification statistic is seeded (every row seen once, |dL/d(u, v)| uniform in [0, 0.04]
    px, so about half the rows pass gamma_g = 0.02 and, at the new splats' size, are
    duplicated).  Wall times, host-synchronous (ags_map_lifecycle reads its counts back)."""
    import torch
    from paper_2510_26358_amd.rasterizer import LifecycleParams
    n = gm.n
    count = torch.ones(n, device="cuda")
    accum = torch.rand(n, device="cuda", generator=gen) * 0.04
    noise = torch.randn(n, 2, 3, device="cuda", generator=gen)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    acts, c, _ = gm.lifecycle(ras, LifecycleParams(do_prune=True, do_densify=True, do_reset=False),
                              stats=(accum, count), noise=noise)
    life_ms = (time.perf_counter() - w0) * 1e3
    pts = torch.rand(1 << 16, 3, device="cuda", generator=gen) * 3.0
    cols = torch.rand(1 << 16, 3, device="cuda", generator=gen)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    _, c2 = gm.insert(pts, cols, frame)
    ins_ms = (time.perf_counter() - w0) * 1e3
    gm.sync()
    return {"rows_in": n, "rows_out": c["n_resident"], "new_ids": c["n_new"], "retired": c["n_retired"],
            "ms_wall": round(life_ms, 4), "next_insert_points": 1 << 16, "next_insert_ms_wall": round(ins_ms, 4),
            "next_insert_evicted": c2["n_evicted"], "resident_after": c2["n_resident"]}


def per_view_loop(ras, p, cams, views, tg, grads, loss, steps, warmup):
    """The comparator: the same kernels launched once per view in a host loop (each view its
    own projection, binning and sorts; gradients accumulated across views; eager launches)."""
    import torch
    from paper_2510_26358_amd.rasterizer import LossTargets
    per = []
    pb = views.pix_base
    for b in range(views.n_views):
        vb = views.subset(b)
        cb = cams[b:b + 1].contiguous()
        capb, _, _ = calibrate(ras, p, cb, vb)
        bb = ras.buffers(vb, p.n, p.sh_degree, capb)
        ob = ras.outputs(vb)
        o0, o1 = tg.depth_offsets[b], tg.depth_offsets[b + 1]
        tgb = LossTargets(tg.gt_rgb[3 * pb[b]:3 * pb[b + 1]], None, [tg.l1_count[b]], tg.depth_pix[o0:o1],
                          tg.depth_val[o0:o1], tg.depth_sigma[o0:o1], [0, o1 - o0], tg.w_l1, tg.lambda_lidar)
        per.append((vb, cb, bb, ob, tgb, torch.zeros(1, 6, device="cuda")))

    def loop_step():
        for b, (vb, cb, bb, ob, tgb, pz) in enumerate(per):
            ras.forward_into(p, cb, vb, bb, ob)
            ras.backward_into(p, cb, vb, bb, ob, grads, pz, loss=tgb, loss_out=loss, accumulate=b > 0)

    t = time_steps(loop_step, steps, warmup)
    tr = time_trials(loop_step, steps)
    del per
    return t, tr


def capture(step, warmup):
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    return g


def measure_workload(name, args, loop=True, px_per_view=0):
    """A further workload of the configuration table as a sub-record of the bench line: its
    own autotuned launch shapes, the graph-captured batched step (for `refine` the whole
    refinement step: forward, backward with Adam fused in, pose update), the per-view loop
    where asked, and oracle parity on a seeded pixel sample in the timed configuration."""
    import torch
    from paper_2510_26358_amd.rasterizer import Rasterizer
    from paper_2510_26358_amd.tune import tune
    t0 = time.perf_counter()
    sc = make_workload(name)
    ras = Rasterizer(0)
    p, cams, views, tg = setup(sc, ras)
    tuned = tune(ras, p, cams, views, tg, use_cache=False)
    cap, K, V = calibrate(ras, p, cams, views)
    P = views.n_pixels
    rec = {"workload": sc.name, "n_gaussians": sc.n, "views": views.n_views, "pixels": P,
           "resolution": sorted({f"{w}x{h}" for w, h in zip(views.widths, views.heights)}),
           "launch": tuned["best"], "visible_pairs": V, "intersections": K}
    grads = p.zeros_like()
    pose = torch.zeros(views.n_views, 6, device="cuda")
    loss = torch.zeros(1, device="cuda")
    if name == "refine":
        from paper_2510_26358_amd.refine import Refiner
        # parity first: the refinement step updates the parameters in place
        if px_per_view:
            rec["parity"], _ = oracle_leg(sc, ras, px_per_view, seed=6)
        refiner = Refiner(ras, p, cams, views, tg, capacity=cap)
        step = refiner.step
        rec["step"] = "forward + fused-loss backward with Adam fused in + pose Adam and retraction (graph)"
    else:
        buf = ras.buffers(views, p.n, p.sh_degree, cap)
        out = ras.outputs(views)

        def step():
            ras.forward_into(p, cams, views, buf, out)
            ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss)
        rec["step"] = "forward + fused-loss backward (graph)"
    g = capture(step, args.warmup)
    t = time_steps(g.replay, args.steps, args.warmup)
    rec["ms_per_step"] = round(t * 1e3, 4)
    rec["value"] = round(P / t / 1e6, 2)
    rec["timing_rule"] = time_trials(g.replay, args.steps)
    if name == "refine":
        assert refiner.check_capacity(), "capacity overflow during timing"
    if loop and views.n_views > 1 and name != "refine":
        t_l, tr_l = per_view_loop(ras, p, cams, views, tg, grads, loss, args.steps, args.warmup)
        rec["per_view_loop"] = {"value": round(P / t_l / 1e6, 2), "ms_per_step": round(t_l * 1e3, 4),
                                "speedup_batched": round(t_l / t, 3),
                                "speedup_batched_median": round(tr_l["median_ms"] / rec["timing_rule"]["median_ms"], 3),
                                "timing_rule": tr_l}
    if px_per_view and name != "refine":
        rec["parity"], _ = oracle_leg(sc, ras, px_per_view, seed=6)
    rec["wall_s"] = round(time.perf_counter() - t0, 1)
    log(f"[bench] {sc.name}: {rec['ms_per_step']} ms/step, {rec['value']} Mpixel/s "
        f"{'(loop speedup ' + str(rec['per_view_loop']['speedup_batched']) + 'x) ' if 'per_view_loop' in rec else ''}"
        f"parity {rec.get('parity', {}).get('pass')}")
    del g, p, grads, sc
    if name != "refine":
        del buf, out
    torch.cuda.empty_cache()
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="multi_view")
    ap.add_argument("--tile", default="auto", help="8, 16, 32 or auto (autotuner)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--ppt", type=int, default=1)
    ap.add_argument("--batch-bwd", type=int, default=0)
    ap.add_argument("--ppt-bwd", type=int, default=0)
    ap.add_argument("--no-loop", action="store_true", help="skip the per-view loop comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (parity + CPU baseline)")
    ap.add_argument("--oracle-px", type=int, default=2048,
                    help="seeded pixels per view of the oracle leg (parity and CPU baseline)")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of a HIP graph")
    ap.add_argument("--ssim", type=float, default=0.2,
                    help="also time the step with the D-SSIM part of L_3DGS at this weight (0: skip)")
    ap.add_argument("--rendered-variance", type=float, default=1e-4, metavar="FLOOR",
                    help="also time the step with the rendered-variance LiDAR term (this variance floor, "
                         "m^2; 0: skip)")
    ap.add_argument("--lifecycle", type=int, default=1,
                    help="also time the step accumulating the densification statistic and one lifecycle "
                         "pass (prune / split / duplicate / reset) over the Gaussians (0: skip)")
    ap.add_argument("--voxel-map", type=int, default=1,
                    help="also time voxel-map insertion calls (2^20 points each, resident bound 2^20; 0: skip)")
    ap.add_argument("--sub-workloads", default="submaps,refine",
                    help="further workloads reported as sub-records of the line (comma list; '' for none)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); sharding the path across "
              f"GPUs is described, not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2510_26358_amd.rasterizer import Rasterizer

    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {4 * n} bytes read and written")
        del src, dst
    t0 = time.perf_counter()
    sc = make_workload(args.workload)
    log(f"[bench] workload {sc.name}: N={sc.n}, views={len(sc.cameras)}, P={sc.n_pixels} "
        f"(generated in {time.perf_counter() - t0:.1f}s)")
    auto = args.tile == "auto"
    ras = Rasterizer(0, tile=16 if auto else int(args.tile), batch=args.batch, px_per_thread=args.ppt,
                     batch_bwd=args.batch_bwd, px_per_thread_bwd=args.ppt_bwd)
    p, cams, views, tg = setup(sc, ras)
    tuned = None
    if auto:
        from paper_2510_26358_amd.tune import tune
        tuned = tune(ras, p, cams, views, tg, use_cache=False, log=log)
        log(f"[bench] autotuner picked tile/batch/ppt = {tuned['best']}")
    tile, batch, ppt = ras.cfg.tile, ras.cfg.batch, ras.cfg.px_per_thread
    batch_b = ras.cfg.batch_bwd or batch
    ppt_b = ras.cfg.px_per_thread_bwd or ppt
    cap, K, V = calibrate(ras, p, cams, views)
    log(f"[bench] V={V} visible pairs, K={K} intersections, capacity {cap}")
    buf = ras.buffers(views, p.n, p.sh_degree, cap)
    out = ras.outputs(views)
    grads = p.zeros_like()
    pose = torch.zeros(views.n_views, 6, device="cuda")
    loss = torch.zeros(1, device="cuda")
    refiner = None
    if args.workload == "refine":
        from paper_2510_26358_amd.refine import Refiner
        refiner = Refiner(ras, p, cams, views, tg, capacity=cap)

        def step():
            refiner.step()
    else:
        def step():
            ras.forward_into(p, cams, views, buf, out)
            ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss)

    t_eager = None
    if refiner is None:
        t_eager = time_steps(step, args.steps, args.warmup)
        log(f"[bench] batched (eager launches): {t_eager * 1e3:.3f} ms/step")
    timed = step
    if not args.no_graph:
        timed = capture(step, args.warmup).replay
    t_b = time_steps(timed, args.steps, args.warmup)
    rule = time_trials(timed, args.steps)
    P = views.n_pixels
    mpx = P / t_b / 1e6
    lval = (refiner.loss if refiner is not None else loss).item()
    log(f"[bench] batched{' (graph)' if not args.no_graph else ''}: {t_b * 1e3:.3f} ms/step, {mpx:.1f} Mpixel/s, "
        f"loss {lval:.5f}; {rule}")
    over_buf = refiner.buf if refiner is not None else buf
    assert over_buf.counters()[2] == 0, "capacity overflow during timing"
    n_listed = over_buf.n_listed()

    # per-stage times over a second timed pass with events enabled
    roof, info = None, None
    if not args.no_profile:
        ras.profile(True)
        ras.profile_reset()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        prof = ras.profile_read()
        ras.profile(False)
        stage_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items() if v[1] > 0}
        log(f"[bench] per-stage avg ms: {stage_ms}")
        launch = {"raster_bwd": (tile, ppt_b, batch_b), "raster_fwd": (tile, ppt, batch)}
        top = max((k for k, v in prof.items() if v[1] > 0), key=lambda k: prof[k][0])
        roof, info = dominant_roofline(prof, views, over_buf, over_buf.sizes, args.steps, p.n,
                                       (p.sh_degree + 1) ** 2, args.workload, launch.get(top))
        info["stage_ms"] = stage_ms
        info["stages"] = stage_rooflines(stage_ms, info["pairs_evaluated"], P, p.n, (p.sh_degree + 1) ** 2,
                                         over_buf.sizes.n_pairs, info["V"], info["K"],
                                         int(tg.depth_pix.numel()), t_b * 1e3,
                                         fused_adam=refiner is not None and refiner.fused_adam)
        roof["step_hbm_frac"] = info["stages"]["step"]["frac"]

    # the same step with the D-SSIM part of the photometric loss switched on
    with_ssim = None
    if args.ssim > 0 and refiner is None:
        tg.ssim_weight = args.ssim
        timed_s = capture(step, args.warmup).replay if not args.no_graph else step
        t_s = time_steps(timed_s, args.steps, args.warmup)
        with_ssim = {"ssim_weight": args.ssim, "ms_per_step": round(t_s * 1e3, 4),
                     "value": round(P / t_s / 1e6, 2), "loss": round(loss.item(), 6)}
        if not args.no_profile:
            ras.profile(True)
            ras.profile_reset()
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            pr = ras.profile_read()
            ras.profile(False)
            if pr.get("ssim", (0, 0))[1]:
                ms = pr["ssim"][0] / pr["ssim"][1]
                achieved = SSIM_FLOP_PER_PIXEL_CHANNEL * 3 * P / (ms * 1e-3) / 1e12
                with_ssim["ssim_stage_ms"] = round(ms, 4)
                with_ssim["ssim_roofline"] = {
                    "bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                    "frac_nonpacked": round(achieved / FP32_NONPACKED_TFLOPS, 4),
                    "work": f"{3 * P} pixel-channels x {SSIM_FLOP_PER_PIXEL_CHANNEL} FLOP"}
        log(f"[bench] with D-SSIM (weight {args.ssim}): {t_s * 1e3:.3f} ms/step, {P / t_s / 1e6:.1f} Mpixel/s")
        tg.ssim_weight = 0.0

    # the same step with the rendered-variance reading of the LiDAR term
    with_rv = None
    if args.rendered_variance > 0 and refiner is None:
        out_v = ras.outputs(views, depth_var=True)
        tg.sigma_mode, tg.sigma_floor = "rendered", args.rendered_variance

        def step_v():
            ras.forward_into(p, cams, views, buf, out_v)
            ras.backward_into(p, cams, views, buf, out_v, grads, pose, loss=tg, loss_out=loss)

        timed_v = capture(step_v, args.warmup).replay if not args.no_graph else step_v
        t_v = time_steps(timed_v, args.steps, args.warmup)
        with_rv = {"sigma_floor": args.rendered_variance, "ms_per_step": round(t_v * 1e3, 4),
                   "value": round(P / t_v / 1e6, 2), "loss": round(loss.item(), 6)}
        log(f"[bench] with the rendered-variance LiDAR term: {t_v * 1e3:.3f} ms/step, {P / t_v / 1e6:.1f} Mpixel/s")
        tg.sigma_mode = "fixed"
        del out_v

    lifecycle = None
    if args.lifecycle and refiner is None:
        lifecycle = measure_lifecycle(ras, p, cams, views, buf, out, grads, pose, tg, loss, args, t_b)

    vmap = None
    if args.voxel_map and refiner is None:
        vmap = measure_voxel_map(ras, args)

    loop = None
    if not args.no_loop and views.n_views > 1 and refiner is None:
        t_l, tr_l = per_view_loop(ras, p, cams, views, tg, grads, loss, args.steps, args.warmup)
        loop = {"value": round(P / t_l / 1e6, 2), "ms_per_step": round(t_l * 1e3, 4),
                "speedup_batched": round(t_l / t_b, 3),
                "speedup_batched_eager": round(t_l / t_eager, 3) if t_eager else None,
                "speedup_batched_median": round(tr_l["median_ms"] / rule["median_ms"], 3),
                "timing_rule": tr_l}
        log(f"[bench] per-view loop: {t_l * 1e3:.3f} ms/step, {P / t_l / 1e6:.1f} Mpixel/s "
            f"(batched speedup {t_l / t_b:.2f}x)")

    parity, cpu = None, None
    if not args.no_cpu:
        log("[bench] oracle leg: parity of the timed configuration on a seeded sample, and the FP64 oracle's "
            "time on the host...")
        parity, cpu = oracle_leg(sc, ras, args.oracle_px, single_thread_px=512)
        cpu["other_configs"] = oracle_other_configs()
        log(f"[bench] parity {parity}")
        log(f"[bench] cpu oracle: {cpu}")

    del buf, out, grads, refiner, over_buf, timed, step
    torch.cuda.empty_cache()
    subs = {}
    for name in [w for w in args.sub_workloads.split(",") if w and w != args.workload]:
        subs[name] = measure_workload(name, args, loop=not args.no_loop,
                                      px_per_view=0 if args.no_cpu else (256 if name == "submaps" else 1024))

    rec = {
        "metric": METRIC, "value": round(mpx, 2), "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_b * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "timing": "HIP graph replay" if not args.no_graph else "eager launches",
        "timing_rule": rule,
        "ms_per_step_eager": round(t_eager * 1e3, 4) if t_eager else None,
        "data": "synthetic",
        "config": {"workload": sc.name, "n_gaussians": sc.n, "views": views.n_views,
                   "resolution": [[w, h] for w, h in zip(views.widths, views.heights)],
                   "pixels": P, "sh_degree": sc.sh_degree, "loss": "L1 + LiDAR KL",
                   "tile": tile, "lds_batch": batch, "px_per_thread": ppt, "lds_batch_bwd": batch_b,
                   "px_per_thread_bwd": ppt_b,
                   "autotuned": None if tuned is None else tuned["ms"],
                   "visible_pairs": V, "intersections": K, "tile_list_entries": n_listed},
        "per_view_loop": loop, "parity": parity, "roofline": roof, "dominant": info, "cpu_baseline": cpu,
        "workloads": subs,
        "with_ssim": with_ssim, "with_rendered_variance": with_rv, "lifecycle": lifecycle,
        "voxel_map": vmap,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
