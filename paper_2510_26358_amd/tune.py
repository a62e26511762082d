"""Autotuner for the raster launch shape: tile edge T, Gaussians per LDS batch M and pixels
per thread, chosen by timing a full forward + backward step of the caller's workload.

Results are cached in a JSON file keyed by device name and workload shape (number of
Gaussians, SH degree, view sizes), so a shape is tuned once per machine.  The tile size
changes the binning, so every candidate recalibrates its intersection capacity.
"""
from __future__ import annotations

import json
import os
import time

import torch

# (tile, batch, pixels per thread): the launch shapes compiled into the library
CANDIDATES = [(8, 64, 1), (8, 128, 1), (16, 128, 1), (16, 256, 1), (16, 128, 2), (16, 256, 2),
              (16, 64, 4), (32, 256, 4), (32, 512, 2)]


def _cache_path():
    base = os.environ.get("AGS_TUNE_CACHE") or os.path.join(
        os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "agsplat", "tune.json")
    return base


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


def time_config(ras, params, cams, views, targets, tile, batch, ppt, steps=5, warmup=2, headroom=1.15):
    """ms per fwd+bwd step for one launch shape (the context is left in that shape)."""
    ras.set_config(tile=tile, batch=batch, px_per_thread=ppt)
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
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3, k


def tune(ras, params, cams, views, targets, candidates=CANDIDATES, steps=5, warmup=2, use_cache=True,
         log=None):
    """Time every candidate launch shape; set the fastest on `ras` and return
    {"best": (tile, batch, ppt), "ms": {...}, "cached": bool}."""
    key = shape_key(views, params.n, params.sh_degree)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        best = tuple(cache[key]["best"])
        ras.set_config(tile=best[0], batch=best[1], px_per_thread=best[2])
        return {"best": best, "ms": cache[key]["ms"], "cached": True}
    results = {}
    for (t, m, p) in candidates:
        ms, k = time_config(ras, params, cams, views, targets, t, m, p, steps, warmup)
        results[f"T{t}_M{m}_P{p}"] = round(ms, 4)
        if log:
            log(f"[tune] tile {t} batch {m} ppt {p}: {ms:.3f} ms/step (K={k})")
    best_name = min(results, key=results.get)
    best = next(c for c in candidates if f"T{c[0]}_M{c[1]}_P{c[2]}" == best_name)
    ras.set_config(tile=best[0], batch=best[1], px_per_thread=best[2])
    if use_cache:
        cache[key] = {"best": list(best), "ms": results}
        _store_cache(cache)
    return {"best": best, "ms": results, "cached": False}
