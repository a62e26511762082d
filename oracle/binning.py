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
  tile rectangle: x_lo // T .. x_hi // T, y_lo // T .. y_hi // T (the candidate tiles)
  a candidate tile is kept when the alpha >= alpha_min ellipse reaches the rectangle of its
      pixel centres [x0 + 1/2, x1 - 1/2] x [y0 + 1/2, y1 - 1/2] (clipped to the image):
      with d = pixel centre - (u, v) and Q(d) = a dx^2 + 2 b dx dy + c dy^2 (the conic), the
      minimum of Q over that rectangle is at most tau2 = 1.001 ex^2 (a c - b^2) / c + 0.001
      (ex^2 (a c - b^2) / c is the level 2 ln(o / alpha_min) whose bounding box has the
      half-width ex; the margin keeps the test conservative under rounding).  The minimum is
      0 when the centre lies inside, else it lies at a corner or at an edge's interior
      minimiser (tested without division, see `tile_reached`); every step is one rounded
      float32 operation in the order written there, so the decision is reproducible bit for
      bit.
  (`tile_min_q_f64` / `membership_f64` state the same rule in float64 for the independent
  gate: the float32 steps decide only candidates within rounding of the level)
  one intersection per (view b, Gaussian i, kept tile) with global tile id
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


_F = np.float32


def tile_tau2(a, b, c, ex):
    """1.001 ex^2 (a c - b^2) / c + 0.001, each step rounded to float32."""
    a, b, c, ex = (np.asarray(x, np.float32) for x in (a, b, c, ex))
    det = a * c - b * b
    t = (ex * ex) * det / c
    return t * _F(1.001) + _F(1e-3)


def _q(a, b, c, x, y):
    """a x^2 + 2 b x y + c y^2 in float32 steps."""
    return ((a * x) * x + ((_F(2) * b) * x) * y) + (c * y) * y


def tile_reached(u, v, a, b, c, tau2, tx, ty, T, W, H):
    """Whether the ellipse Q(d) <= tau2 reaches the pixel centres of tile (tx, ty): the centre
    inside the rectangle, a corner with Q <= tau2, or an edge whose interior holds the
    quadratic's minimiser along it with that minimum, X^2 (a c - b^2) / c (for x = X),
    at most tau2 -- compared as X^2 det <= tau2 c, so that no step divides.  Arrays
    broadcast; float32 steps; a NaN keeps the tile."""
    u, v, a, b, c, tau2 = (np.asarray(x, np.float32) for x in (u, v, a, b, c, tau2))
    tx = np.asarray(tx, np.int64)
    ty = np.asarray(ty, np.int64)
    X0 = (tx * T).astype(np.float32) + _F(0.5)
    X1 = np.minimum((tx + 1) * T, W).astype(np.float32) - _F(0.5)
    Y0 = (ty * T).astype(np.float32) + _F(0.5)
    Y1 = np.minimum((ty + 1) * T, H).astype(np.float32) - _F(0.5)
    lx, hx, ly, hy = X0 - u, X1 - u, Y0 - v, Y1 - v
    det = a * c - b * b
    with np.errstate(all="ignore"):
        hit = (lx <= 0) & (hx >= 0) & (ly <= 0) & (hy >= 0)
        for x in (lx, hx):
            for y in (ly, hy):
                hit = hit | ~(_q(a, b, c, x, y) > tau2)
        for X in (lx, hx):       # edges x = X: minimiser y = -b X / c inside [ly, hy]
            m = -(b * X)
            hit = hit | ((c * ly <= m) & (m <= c * hy) & ~((X * X) * det > tau2 * c))
        for Y in (ly, hy):       # edges y = Y: minimiser x = -b Y / a inside [lx, hx]
            m = -(b * Y)
            hit = hit | ((a * lx <= m) & (m <= a * hx) & ~((Y * Y) * det > tau2 * a))
    return hit


def tile_min_q_f64(u, v, a, b, c, tx, ty, T, W, H):
    """Float64 minimum of Q(d) = a dx^2 + 2 b dx dy + c dy^2 over the pixel centres' rectangle
    of tile (tx, ty), d = point - (u, v): zero when (u, v) lies inside, else the least of the
    four edge minima (on an edge the quadratic is a parabola whose minimiser is clipped to
    the edge).  Independent of the float32 decision rule of `tile_reached`: the plain
    geometric statement that rule approximates."""
    u, v, a, b, c = (float(x) for x in (u, v, a, b, c))
    lx = tx * T + 0.5 - u
    hx = min((tx + 1) * T, W) - 0.5 - u
    ly = ty * T + 0.5 - v
    hy = min((ty + 1) * T, H) - 0.5 - v
    if lx <= 0.0 <= hx and ly <= 0.0 <= hy:
        return 0.0

    def q(x, y):
        return a * x * x + 2.0 * b * x * y + c * y * y

    best = np.inf
    for X in (lx, hx):
        y = min(max(-b * X / c, ly), hy)
        best = min(best, q(X, y))
    for Y in (ly, hy):
        x = min(max(-b * Y / a, lx), hx)
        best = min(best, q(x, Y))
    return best


def tile_level_f64(a, b, c, ex):
    """1.001 ex^2 (a c - b^2) / c + 0.001 in float64."""
    a, b, c, ex = (float(x) for x in (a, b, c, ex))
    return 1.001 * ex * ex * (a * c - b * b) / c + 0.001


def membership_f64(records, views, T: int, rel=1e-4):
    """Tile membership by the float64 statement of the tile rule: the candidate tiles of each
    valid record's footprint rectangle (`pixel_rect_f32`) whose float64 minimum of Q
    (`tile_min_q_f64`) is at most the float64 level.  Returns (kept, ambiguous): sets of
    (global tile, Gaussian index); a candidate whose minimum lies within rel (relative) of
    the level is ambiguous -- float32 rounding may decide it either way."""
    kept, amb = set(), set()
    base = 0
    for (W, H, g0), rec in zip(views, records):
        ntx, nty = tile_grid(W, H, T)
        x0, y0, x1, y1, ne = pixel_rect_f32(rec["u"], rec["v"], rec["ex"], rec["ey"], W, H)
        ok = ne & np.asarray(rec["valid"], bool)
        for i in np.nonzero(ok)[0]:
            lev = tile_level_f64(rec["a"][i], rec["b"][i], rec["c"][i], rec["ex"][i])
            for ty in range(y0[i] // T, y1[i] // T + 1):
                for tx in range(x0[i] // T, x1[i] // T + 1):
                    m = tile_min_q_f64(rec["u"][i], rec["v"][i], rec["a"][i], rec["b"][i], rec["c"][i],
                                       tx, ty, T, W, H)
                    key = (base + ty * ntx + tx, g0 + int(i))
                    if abs(m - lev) <= rel * max(1.0, lev):
                        amb.add(key)
                    elif m <= lev:
                        kept.add(key)
        base += ntx * nty
    return kept, amb


def bin_reference(records, views, T: int):
    """records: list per view of dict(u, v, a, b, c, ex, ey, z (float32 arrays over the
    view's Gaussian range), valid (bool)); views: list of (width, height, g_begin).

    Returns keys (uint64, sorted, kept intersections), vals (uint32 Gaussian index), ranges
    (n_tiles, 2) uint32, counts per (view, local Gaussian) of candidate tiles (list of int64
    arrays), tile_base (n_views+1)."""
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
        tau2 = tile_tau2(rec["a"], rec["b"], rec["c"], rec["ex"])
        for i in np.nonzero(ok)[0]:
            ty = np.arange(ty0[i], ty1[i] + 1)
            tx = np.arange(tx0[i], tx1[i] + 1)
            TY, TX = np.meshgrid(ty, tx, indexing="ij")
            keep = tile_reached(rec["u"][i], rec["v"][i], rec["a"][i], rec["b"][i], rec["c"][i], tau2[i],
                                TX, TY, T, W, H).ravel()
            tiles = (tile_base[b] + TY * ntx + TX).ravel().astype(np.uint64)[keep]
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
