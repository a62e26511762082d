"""Integer reference for tile binning and the (view, tile, depth) key order (oracle).

The paper's renderer is "standard 3DGS" (Sec. III-B): Gaussians are assigned to the image
tiles their footprint touches and each tile's list is ordered by depth.  This module fixes
that order as a plain definition so the kernel's lists can be compared bit for bit:

  footprint rectangle (pixels) of a projected Gaussian with centre (u, v) and bounding
  half-extents (ex, ey), evaluated in float32 exactly as written (the kernel's precision,
  because the rounding decides an integer):
      x_lo = floor((u - ex) - 0.5), x_hi = ceil((u + ex) - 0.5), clamped to [0, W-1]
      y_lo = floor((v - ey) - 0.5), y_hi = ceil((v + ey) - 0.5), clamped to [0, H-1]
      empty when x_lo > x_hi or y_lo > y_hi (or when the pair is culled)
  tile rectangle: x_lo // T .. x_hi // T, y_lo // T .. y_hi // T
  one intersection per (view b, Gaussian i, tile) with global tile id
      tile_base[b] + ty * ntx_b + tx and key (tile_id << 32) | bits(float32 depth)
  emitted in (b, i, ty, tx) order and stably sorted by key; ranges[tile] = [first, last+1).

Depths are positive (z >= z_near > 0), so the float32 bit pattern orders like the value.
"""
from __future__ import annotations

import numpy as np


def tile_grid(width: int, height: int, T: int):
    return (width + T - 1) // T, (height + T - 1) // T


def pixel_rect_f32(u, v, ex, ey, width, height):
    """Float32 footprint rectangle in pixels; returns (x0, y0, x1, y1, nonempty)."""
    u = np.asarray(u, np.float32)
    v = np.asarray(v, np.float32)
    ex = np.asarray(ex, np.float32)
    ey = np.asarray(ey, np.float32)
    half = np.float32(0.5)
    fx0 = np.floor((u - ex) - half)
    fx1 = np.ceil((u + ex) - half)
    fy0 = np.floor((v - ey) - half)
    fy1 = np.ceil((v + ey) - half)
    # clamp in the float domain before converting (values may be huge)
    x0 = np.clip(fx0, 0, width).astype(np.int64)
    x1 = np.clip(fx1, -1, width - 1).astype(np.int64)
    y0 = np.clip(fy0, 0, height).astype(np.int64)
    y1 = np.clip(fy1, -1, height - 1).astype(np.int64)
    nonempty = (x0 <= x1) & (y0 <= y1)
    return x0, y0, x1, y1, nonempty


def bin_reference(records, views, T: int):
    """records: list per view of dict(u, v, ex, ey, z (float32 arrays over the view's
    Gaussian range), valid (bool)); views: list of (width, height, g_begin).

    Returns keys (uint64, sorted), vals (uint32 Gaussian index), ranges (n_tiles, 2) uint32,
    counts per (view, local Gaussian) (list of int64 arrays), tile_base (n_views+1)."""
    tile_base = [0]
    for (W, H, _g0) in views:
        ntx, nty = tile_grid(W, H, T)
        tile_base.append(tile_base[-1] + ntx * nty)
    keys_l, vals_l, counts = [], [], []
    for b, ((W, H, g0), rec) in enumerate(zip(views, records)):
        ntx, nty = tile_grid(W, H, T)
        x0, y0, x1, y1, ne = pixel_rect_f32(rec["u"], rec["v"], rec["ex"], rec["ey"], W, H)
        ok = ne & np.asarray(rec["valid"], bool)
        tx0, tx1, ty0, ty1 = x0 // T, x1 // T, y0 // T, y1 // T
        cnt = np.where(ok, (tx1 - tx0 + 1) * (ty1 - ty0 + 1), 0)
        counts.append(cnt)
        zbits = np.asarray(rec["z"], np.float32).view(np.uint32).astype(np.uint64)
        for i in np.nonzero(ok)[0]:
            ty = np.arange(ty0[i], ty1[i] + 1)
            tx = np.arange(tx0[i], tx1[i] + 1)
            tiles = (tile_base[b] + ty[:, None] * ntx + tx[None, :]).ravel().astype(np.uint64)
            keys_l.append((tiles << np.uint64(32)) | zbits[i])
            vals_l.append(np.full(len(tiles), g0 + i, np.uint32))
    keys = np.concatenate(keys_l) if keys_l else np.zeros(0, np.uint64)
    vals = np.concatenate(vals_l) if vals_l else np.zeros(0, np.uint32)
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    vals = vals[order]
    n_tiles = tile_base[-1]
    ranges = np.zeros((n_tiles, 2), np.uint32)
    if len(keys):
        tiles = (keys >> np.uint64(32)).astype(np.int64)
        starts = np.searchsorted(tiles, np.arange(n_tiles), side="left")
        ends = np.searchsorted(tiles, np.arange(n_tiles), side="right")
        ranges[:, 0] = np.where(ends > starts, starts, 0)
        ranges[:, 1] = np.where(ends > starts, ends, 0)
    return keys, vals, ranges, counts, np.array(tile_base, np.int64)
