"""Autotuner front end for the raster launch shapes: tile edge T (shared by binning, forward
and backward), and for each raster kernel its Gaussians per LDS batch and pixels per thread.

The search runs in the library (`ags_tune`): for every tile size and every launch shape
compiled for it, a few full forward + backward steps of the caller's workload are timed with
per-stage HIP events; the forward and backward shapes are chosen independently (they only
share T) and the tile size with the smallest resulting step time wins.  This module keeps
the host policy: picks are cached in a JSON file keyed by device name and workload shape,
so a shape is tuned once per machine.
"""
from __future__ import annotations

import json
import os

import torch


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


def tune(ras, params, cams, views, targets, steps=4, warmup=2, use_cache=True, log=None):
    """Choose and set the fastest tile size and per-kernel launch shapes with the library's
    autotuner (`ags_tune`: the search and its timing run behind the C ABI), caching the pick
    per device and workload shape.  Returns {"best": {...}, "ms": {...}, "cached": bool}."""
    import ctypes as C
    from . import _lib as L
    key = shape_key(views, params.n, params.sh_degree)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        _apply(ras, cache[key]["best"])
        return {"best": cache[key]["best"], "ms": cache[key]["ms"], "cached": True}
    best = L.Config()
    pred = C.c_float()
    entries = (L.TuneEntry * 32)()
    n_rep = C.c_int32()
    g = params.c()
    lc = targets.c()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = ras.lib.ags_tune(ras.ctx, C.byref(views.c), C.byref(g), C.c_void_p(cams.data_ptr()), C.byref(lc), steps,
                          warmup, C.byref(best), C.byref(pred), entries, 32, C.byref(n_rep), stream)
    L.check(rc, "ags_tune", ras.ctx)
    table = {}
    for e in entries[:min(n_rep.value, 32)]:
        table[f"T{e.tile}_M{e.batch}_P{e.px_per_thread}"] = {
            "step_ms": round(e.step_ms, 4), "raster_fwd": round(e.raster_fwd_ms, 4),
            "raster_bwd": round(e.raster_bwd_ms, 4), "K": int(e.intersections)}
        if log:
            log(f"[tune] tile {e.tile} batch {e.batch} ppt {e.px_per_thread}: step {e.step_ms:.3f} ms, "
                f"fwd {e.raster_fwd_ms:.3f}, bwd {e.raster_bwd_ms:.3f} (K={e.intersections})")
    pick = {"tile": best.tile, "batch": best.batch, "ppt": best.px_per_thread, "batch_bwd": best.batch_bwd,
            "ppt_bwd": best.px_per_thread_bwd, "predicted_step_ms": round(pred.value, 4)}
    # ags_tune already set the pick on the context; keep the binding's copy in step
    ras.cfg = best
    if use_cache:
        cache[key] = {"best": pick, "ms": table}
        _store_cache(cache)
    return {"best": pick, "ms": table, "cached": False}
