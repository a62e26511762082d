"""Autotuner for the raster launch shapes: tile edge T (shared by binning, forward and
backward), and for each raster kernel its Gaussians per LDS batch and pixels per thread.

For every tile size and every launch shape compiled for it, a few full forward + backward
steps of the caller's workload are timed with the library's per-stage HIP events; the
forward and backward shapes are then chosen independently (they only share T) and the tile
size with the smallest resulting step time wins.  Results are cached in a JSON file keyed
by device name and workload shape, so a shape is tuned once per machine.  The tile size
changes the binning, so every tile size recalibrates its intersection capacity.
"""
from __future__ import annotations

import json
import os
import time

import torch

# (batch, pixels per thread) launch shapes compiled for each tile size
SHAPES = {8: [(64, 1), (128, 1)],
          16: [(128, 1), (256, 1), (128, 2), (256, 2), (64, 4)],
          32: [(256, 4), (512, 2)]}


def _cache_path():
    return os.environ.get("AGS_TUNE_CACHE") or os.path.join(
        os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "agsplat", "tune.json")


def shape_key(views, n, sh_degree):
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    vs = ",".join(f"{w}x{h}:{g1 - g0}" for w, h, g0, g1 in
                  zip(views.widths, views.heights, views.g_begin, views.g_end))
    return f"{dev}|n={n}|deg={sh_degree}|{vs}"


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass


def _apply(ras, best):
    ras.set_config(tile=best["tile"], batch=best["batch"], px_per_thread=best["ppt"],
                   batch_bwd=best["batch_bwd"], px_per_thread_bwd=best["ppt_bwd"])


def time_shape(ras, params, cams, views, targets, tile, batch, ppt, steps=4, warmup=2, headroom=1.15):
    """Per-stage ms of a fwd+bwd step with one launch shape for both raster kernels."""
    ras.set_config(tile=tile, batch=batch, px_per_thread=ppt, batch_bwd=0, px_per_thread_bwd=0)
    out, buf = ras.render(params, cams, views)
    k = int(buf.counters()[0])
    buf = ras.buffers(views, params.n, params.sh_degree, int(k * headroom) + 4096)
    out = ras.outputs(views)
    grads = params.zeros_like()
    pose = torch.zeros(views.n_views, 6, device=params.means.device)
    loss = torch.zeros(1, device=params.means.device)

    def step():
        ras.forward_into(params, cams, views, buf, out)
        ras.backward_into(params, cams, views, buf, out, grads, pose, loss=targets, loss_out=loss)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ras.profile(True)
    ras.profile_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    prof = ras.profile_read()
    ras.profile(False)
    stages = {name: tot / steps for name, (tot, cnt) in prof.items() if cnt}
    return wall, stages, k


def tune(ras, params, cams, views, targets, tiles=(8, 16, 32), steps=4, warmup=2, use_cache=True, log=None):
    """Choose and set the fastest tile size and per-kernel launch shapes.  Returns
    {"best": {...}, "ms": {...}, "cached": bool}."""
    key = shape_key(views, params.n, params.sh_degree)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        _apply(ras, cache[key]["best"])
        return {"best": cache[key]["best"], "ms": cache[key]["ms"], "cached": True}
    table, best, best_total = {}, None, float("inf")
    for t in tiles:
        per = []
        for (m, p) in SHAPES[t]:
            wall, st, k = time_shape(ras, params, cams, views, targets, t, m, p, steps, warmup)
            table[f"T{t}_M{m}_P{p}"] = {"step_ms": round(wall, 4), "raster_fwd": round(st.get("raster_fwd", 0), 4),
                                        "raster_bwd": round(st.get("raster_bwd", 0), 4), "K": k}
            per.append(((m, p), wall, st))
            if log:
                log(f"[tune] tile {t} batch {m} ppt {p}: step {wall:.3f} ms, fwd {st.get('raster_fwd', 0):.3f}, "
                    f"bwd {st.get('raster_bwd', 0):.3f} (K={k})")
        f_best = min(per, key=lambda e: e[2].get("raster_fwd", 0))
        b_best = min(per, key=lambda e: e[2].get("raster_bwd", 0))
        base = per[0]
        rest = base[1] - base[2].get("raster_fwd", 0) - base[2].get("raster_bwd", 0)
        total = rest + f_best[2].get("raster_fwd", 0) + b_best[2].get("raster_bwd", 0)
        if total < best_total:
            best_total = total
            best = {"tile": t, "batch": f_best[0][0], "ppt": f_best[0][1], "batch_bwd": b_best[0][0],
                    "ppt_bwd": b_best[0][1], "predicted_step_ms": round(total, 4)}
    _apply(ras, best)
    if use_cache:
        cache[key] = {"best": best, "ms": table}
        _store_cache(cache)
    return {"best": best, "ms": table, "cached": False}
