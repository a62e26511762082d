"""Pins for the oracle's tile-binning reference (the depth-ordered per-tile lists of the
"standard 3DGS" renderer, Sec. III-B) and for its Adam / se(3) pose update (the joint
refinement of splats and poses, Sec. III-C)."""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

import scipy.optimize

from oracle.binning import bin_reference, pixel_rect_f32, tile_grid, tile_reached, tile_tau2
from oracle.geometry import se3_exp, skew
from oracle.optim import adam_update, pose_update
from oracle.render import leaves, project, render
from oracle.settings import RenderSettings
from paper_2510_26358_amd.scenes import tiny_scene


def _random_records(rng, n, W, H):
    """Seeded projected Gaussians: centre, a random positive-definite screen covariance
    (conic = its inverse), opacity, and the footprint half-widths of the alpha = 1/255 level
    (so that the tile test prunes the rectangle's corners)."""
    u = rng.uniform(-40, W + 40, n).astype(np.float32)
    v = rng.uniform(-40, H + 40, n).astype(np.float32)
    sx = rng.exponential(4.0, n) + 0.3
    sy = rng.exponential(4.0, n) + 0.3
    rho = rng.uniform(-0.95, 0.95, n)
    cxx, cyy, cxy = sx * sx, sy * sy, rho * sx * sy
    det = cxx * cyy - cxy * cxy
    o = rng.uniform(0.01, 0.99, n)
    tau = 2 * np.log(255 * o)
    a, b, c = (cyy / det).astype(np.float32), (-cxy / det).astype(np.float32), (cxx / det).astype(np.float32)
    ex = np.sqrt(tau * cxx).astype(np.float32)
    ey = np.sqrt(tau * cyy).astype(np.float32)
    # quantised depths so that exact key ties occur and stability matters
    z = (np.round(rng.uniform(0.5, 3.0, n) * 8) / 8).astype(np.float32)
    valid = rng.uniform(size=n) > 0.2
    return {"u": u, "v": v, "a": a, "b": b, "c": c, "ex": ex, "ey": ey, "z": z, "valid": valid,
            "o": o.astype(np.float32)}


def _box_min(a, b, c, lo, hi):
    """min of d^T K d over the box lo <= d <= hi (K = [[a, b], [b, c]]) in float64, as the
    bounded least-squares problem min |L^T d|^2 (K = L L^T) solved by scipy."""
    K = np.array([[a, b], [b, c]], np.float64)
    L = np.linalg.cholesky(K)
    r = scipy.optimize.lsq_linear(L.T, np.zeros(2), bounds=(lo, hi), method="bvls")
    d = r.x
    return float(d @ K @ d)


def test_binning_reference_equals_brute_force_enumeration():
    rng = np.random.default_rng(71)
    T = 8
    views = [(64, 40, 0), (50, 30, 300)]
    recs = [_random_records(rng, 300, 64, 40), _random_records(rng, 200, 50, 30)]
    keys, vals, ranges, counts, base = bin_reference(recs, views, T)
    # brute force: every tile of every view that holds a pixel of the footprint rectangle is
    # a candidate; it is kept when the float64 minimum of the conic's quadratic form over its
    # pixel centres (scipy's bounded least squares) is at most 1.001 ex^2 det / c + 0.001.
    # Candidates whose minimum lies within 1e-4 (relative) of that level are ambiguous in
    # float32 and left out of the comparison on both sides.
    items, ambiguous = [], set()
    tile0 = 0
    n_cand = 0
    for b, ((W, H, g0), r) in enumerate(zip(views, recs)):
        ntx, nty = tile_grid(W, H, T)
        for i in range(len(r["u"])):
            if not r["valid"][i]:
                continue
            u, v, ex, ey = (np.float32(r[k][i]) for k in ("u", "v", "ex", "ey"))
            xlo = math.floor(float(np.float32(np.float32(u - ex) - np.float32(0.5))))
            xhi = math.ceil(float(np.float32(np.float32(u + ex) - np.float32(0.5))))
            ylo = math.floor(float(np.float32(np.float32(v - ey) - np.float32(0.5))))
            yhi = math.ceil(float(np.float32(np.float32(v + ey) - np.float32(0.5))))
            A, B, C = (float(r[k][i]) for k in ("a", "b", "c"))
            lev = 1.001 * float(ex) ** 2 * (A * C - B * B) / C + 0.001
            for ty in range(nty):
                for tx in range(ntx):
                    cand = any(xlo <= px <= xhi and ylo <= py <= yhi
                               for py in range(ty * T, min(H, ty * T + T))
                               for px in range(tx * T, min(W, tx * T + T)))
                    if not cand:
                        continue
                    n_cand += 1
                    lo = np.array([tx * T + 0.5 - float(u), ty * T + 0.5 - float(v)])
                    hi = np.array([min(W, tx * T + T) - 0.5 - float(u), min(H, ty * T + T) - 0.5 - float(v)])
                    q = _box_min(A, B, C, lo, hi)
                    tid = tile0 + ty * ntx + tx
                    if abs(q - lev) <= 1e-4 * max(1.0, lev):
                        ambiguous.add((tid, g0 + i))
                    elif q <= lev:
                        zb = int(np.float32(r["z"][i]).view(np.uint32))
                        items.append((((tid) << 32) | zb, g0 + i))
        tile0 += ntx * nty
    items.sort(key=lambda e: e[0])  # Python's sort is stable: ties keep emission order
    assert sum(int(cn.sum()) for cn in counts) == n_cand
    got = [(int(k), int(g)) for k, g in zip(keys, vals) if (int(k) >> 32, int(g)) not in ambiguous]
    assert got == items
    assert len(items) < n_cand  # the test prunes some candidates
    # ranges: every tile's slice holds exactly its keys
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    for t in range(base[-1]):
        s, e = ranges[t]
        assert (tiles[s:e] == t).all()
        assert (e - s) == (tiles == t).sum()


def test_float64_tile_minimum_equals_bounded_least_squares():
    """The closed-form float64 minimum of the conic's quadratic form over a tile's pixel
    centres (interior, else the clipped parabola minima of the four edges) equals scipy's
    bounded least-squares solution on random ellipses and tiles."""
    from oracle.binning import tile_min_q_f64
    rng = np.random.default_rng(73)
    recs = _random_records(rng, 200, 64, 40)
    T, W, H = 8, 64, 40
    n_checked = 0
    for i in range(200):
        A, B, C = (float(recs[k][i]) for k in ("a", "b", "c"))
        for _ in range(4):
            tx, ty = int(rng.integers(0, 8)), int(rng.integers(0, 5))
            got = tile_min_q_f64(recs["u"][i], recs["v"][i], A, B, C, tx, ty, T, W, H)
            lo = np.array([tx * T + 0.5 - float(recs["u"][i]), ty * T + 0.5 - float(recs["v"][i])])
            hi = np.array([min(W, tx * T + T) - 0.5 - float(recs["u"][i]),
                           min(H, ty * T + T) - 0.5 - float(recs["v"][i])])
            ref = _box_min(A, B, C, lo, hi)
            assert abs(got - ref) <= 1e-9 * max(1.0, ref), (i, tx, ty, got, ref)
            n_checked += 1
    assert n_checked == 800


def test_float32_tile_rule_agrees_with_its_float64_statement():
    """The reference's float32 decision steps keep exactly the candidates the float64
    statement keeps, except candidates within 1e-4 (relative) of the level."""
    from oracle.binning import membership_f64
    rng = np.random.default_rng(74)
    T = 8
    views = [(64, 40, 0), (50, 30, 400)]
    recs = [_random_records(rng, 400, 64, 40), _random_records(rng, 300, 50, 30)]
    keys, vals, ranges, counts, base = bin_reference(recs, views, T)
    got = {(int(k) >> 32, int(g)) for k, g in zip(keys, vals)}
    kept, amb = membership_f64(recs, views, T)
    assert kept and (got - amb) == kept


@pytest.mark.parametrize("alpha_min", [1.0 / 255.0, 1e-3, 2e-2])
def test_every_contributing_pixel_lies_in_its_gaussians_tiles(alpha_min):
    """The opacity-aware bounding box, and the ellipse test on its tiles, must cover every
    pixel where the brute-force compositing keeps the Gaussian (alpha >= alpha_min), for each
    tile size and for cutoffs below and above the default 1/255 (the box is the alpha_min
    level of the configured cutoff)."""
    sc = tiny_scene()
    s = RenderSettings(alpha_min=alpha_min)
    out = render(sc, s)[0]
    pr = out["proj"]
    dec = out["dec"]
    W, H = 128, 96
    ext = pr["ext"].numpy()
    x0, y0, x1, y1, ne = pixel_rect_f32(pr["u"].numpy(), pr["v"].numpy(), ext[:, 0], ext[:, 1], W, H)
    con = pr["conic"].detach().numpy().astype(np.float32)
    u32, v32 = pr["u"].detach().numpy().astype(np.float32), pr["v"].detach().numpy().astype(np.float32)
    tau2 = tile_tau2(con[:, 0], con[:, 1], con[:, 2], ext[:, 0].astype(np.float32))
    gi = np.array([i for p in range(W * H) for i in dec.touched[p]], np.int64)
    pp = np.array([p for p in range(W * H) for _ in dec.touched[p]], np.int64)
    px, py = pp % W, pp // W
    assert ne[gi].all()
    for T in (8, 16, 32):
        assert ((x0[gi] // T <= px // T) & (px // T <= x1[gi] // T)).all()
        assert ((y0[gi] // T <= py // T) & (py // T <= y1[gi] // T)).all()
        # the ellipse test keeps the tile of every pixel that uses the Gaussian
        assert tile_reached(u32[gi], v32[gi], con[gi, 0], con[gi, 1], con[gi, 2], tau2[gi], px // T, py // T,
                            T, W, H).all()


def test_adam_matches_torch_adam_in_float64():
    rng = np.random.default_rng(81)
    p0 = rng.normal(size=50)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.normal(size=50)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = adam_update(p, g, m, v, t, 3e-3)
        assert np.allclose(p, tp.detach().numpy(), rtol=0, atol=1e-15)


def test_pose_update_is_left_retraction_of_the_adam_step():
    """First Adam step is -lr * g / (|g| + eps) componentwise; the pose becomes
    expm(hat(delta)) W (matrix exponential of the twist, scipy)."""
    rng = np.random.default_rng(82)
    a = 0.3
    R = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    t = np.array([0.5, -1.0, 2.0])
    g = rng.normal(size=6)
    lr = 1e-2
    R2, t2, m, v = pose_update(R, t, g, np.zeros(6), np.zeros(6), 1, lr)
    delta = -lr * g / (np.abs(g) + 1e-15)
    X = np.zeros((4, 4))
    X[:3, :3] = skew(delta[3:])
    X[:3, 3] = delta[:3]
    E = scipy.linalg.expm(X)
    W = np.eye(4)
    W[:3, :3], W[:3, 3] = R, t
    W2 = E @ W
    assert np.allclose(R2, W2[:3, :3], atol=1e-14) and np.allclose(t2, W2[:3, 3], atol=1e-14)
    assert np.allclose(se3_exp(delta), E, atol=1e-14)
