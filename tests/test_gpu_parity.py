"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Forward: colour / alpha within 1e-4, depth within 1e-4 max(1, D) on every pixel whose result
does not hinge on a decision float32 rounding can flip (flagged by the oracle).  Binning:
bit-exact keys, lists and ranges against the oracle's integer reference on seeded records.
Gradients: 1e-3 relative per tensor, and per element on >= 99.9 % of elements, excluding
Gaussians touched by such decisions.
"""
import numpy as np
import pytest
import torch

from oracle.binning import bin_reference, membership_f64
from oracle.render import loss_and_grads, render
from oracle.settings import RenderSettings
from paper_2510_26358_amd import scenes
from tests.gpu_helpers import (TOL_ALPHA, TOL_DEPTH_REL, TOL_RGB, grad_close, run_forward,
                               run_loss_backward, saved_arrays)
from tests.oracle_helpers import random_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ras():
    from paper_2510_26358_amd.rasterizer import Rasterizer
    return Rasterizer(0)


def _compare_forward(gpu_views, ref_views, scene, pixels=None, max_amb_frac=1e-3):
    for b, (g, r) in enumerate(zip(gpu_views, ref_views)):
        cam = scene.cameras[b]
        pix = r["pix"]
        amb = r["ambiguous"]
        ok = ~amb
        rgb = g["rgb"].reshape(3, -1)[:, pix].T
        dep = g["depth"].reshape(-1)[pix]
        alp = g["alpha"].reshape(-1)[pix]
        e_rgb = np.abs(rgb - r["rgb"])[ok].max(initial=0)
        e_a = np.abs(alp - r["alpha"])[ok].max(initial=0)
        e_d = (np.abs(dep - r["depth"]) / np.maximum(1.0, np.abs(r["depth"])))[ok].max(initial=0)
        print(f"view {b}: {len(pix)} px, ambiguous {amb.sum()}, max err rgb {e_rgb:.2e} alpha {e_a:.2e} "
              f"depth {e_d:.2e}")
        assert amb.mean() <= max_amb_frac + 5.0 / len(pix)
        assert e_rgb <= TOL_RGB and e_a <= TOL_ALPHA and e_d <= TOL_DEPTH_REL


def test_forward_tiny_full_image(ras):
    sc = scenes.tiny_scene()
    gpu, _ = run_forward(sc, ras)
    ref = render(sc, RenderSettings())
    _compare_forward(gpu, ref, sc)


def test_projection_records_match_oracle(ras):
    sc = random_scene(101, n=300, sh_degree=3, n_views=2, width=96, height=64, f=80.0)
    from oracle.render import leaves, project
    _, (p, cams, views, out, buf) = run_forward(sc, ras)
    sv = saved_arrays(buf, views)
    pr = leaves(sc, requires_grad=False)
    base = 0
    for b, cam in enumerate(sc.cameras):
        proj = project(pr, cam, pr["pose_delta"][b], RenderSettings(), sc.sh_degree)
        n = cam.g_end - cam.g_begin
        cnt = sv["pair_count"][base:base + n]
        rec = sv["records"][base:base + n]
        vis = cnt > 0
        valid = proj["valid"].numpy()
        assert not (vis & ~valid).any()
        u = proj["u"].detach().numpy()
        v = proj["v"].detach().numpy()
        con = proj["conic"].detach().numpy()
        ext = proj["ext"].numpy()
        z = proj["z"].detach().numpy()
        o = proj["o"].detach().numpy()
        rgb = proj["rgb"].detach().numpy()
        m = vis
        assert np.allclose(rec[m, 0], u[m], rtol=1e-5, atol=1e-3)
        assert np.allclose(rec[m, 1], v[m], rtol=1e-5, atol=1e-3)
        for j in range(3):
            assert np.allclose(rec[m, 2 + j], con[m, j], rtol=2e-4, atol=1e-6 * np.abs(con[m]).max())
        assert np.allclose(rec[m, 5], o[m], rtol=1e-6, atol=1e-7)
        assert np.allclose(rec[m, 6], z[m], rtol=1e-6)
        assert np.allclose(rec[m, 7], ext[m, 0], rtol=1e-4, atol=1e-4)
        assert np.allclose(rec[m, 8], ext[m, 1], rtol=1e-4, atol=1e-4)
        assert np.allclose(rec[m, 9:12], rgb[m], atol=2e-6)
        base += n


def _synthetic_records(rng, n_views, n, sizes, T, margin=30, keep_frac=0.75):
    """Seeded records: centre (up to `margin` px outside the view), conic of a random
    positive-definite screen covariance, opacity, quantised depth (exact ties) and the
    half-widths of the alpha = 1/255 level; a share `keep_frac` of the pairs is valid."""
    recs, valid, ref_in = [], [], []
    for b in range(n_views):
        W, H = sizes[b]
        u = rng.uniform(-margin, W + margin, n).astype(np.float32)
        v = rng.uniform(-margin, H + margin, n).astype(np.float32)
        sx = rng.exponential(3.0, n) + 0.3
        sy = rng.exponential(3.0, n) + 0.3
        rho = rng.uniform(-0.95, 0.95, n)
        cxx, cyy, cxy = sx * sx, sy * sy, rho * sx * sy
        det = cxx * cyy - cxy * cxy
        o = rng.uniform(0.01, 0.99, n)
        tau = 2 * np.log(255 * o)
        ca, cb, cc = (cyy / det).astype(np.float32), (-cxy / det).astype(np.float32), (cxx / det).astype(np.float32)
        ex = np.sqrt(tau * cxx).astype(np.float32)
        ey = np.sqrt(tau * cyy).astype(np.float32)
        z = (np.round(rng.uniform(0.5, 4.0, n) * 16) / 16).astype(np.float32)  # exact ties
        ok = rng.uniform(size=n) < keep_frac
        r = np.zeros((n, 12), np.float32)
        r[:, 0], r[:, 1], r[:, 2], r[:, 3], r[:, 4] = u, v, ca, cb, cc
        r[:, 5], r[:, 6], r[:, 7], r[:, 8] = o.astype(np.float32), z, ex, ey
        recs.append(r)
        valid.append(ok)
        ref_in.append({"u": u, "v": v, "a": ca, "b": cb, "c": cc, "ex": ex, "ey": ey, "z": z, "valid": ok})
    return np.concatenate(recs), np.concatenate(valid), ref_in


@pytest.mark.parametrize("tile,sizes", [(16, [(128, 96)]), (8, [(70, 45), (33, 17), (128, 64)]),
                                        (32, [(200, 120), (64, 64)]), (16, [(1, 1), (17, 33)]),
                                        (8, [(300, 200), (64, 40)]), (16, [(1280, 800)])])
def test_binning_bit_exact_on_seeded_records(tile, sizes):
    from paper_2510_26358_amd.rasterizer import Rasterizer, ViewSpec
    r = Rasterizer(0, tile=tile, batch=256 if tile != 8 else 64, px_per_thread=1 if tile != 32 else 4)
    rng = np.random.default_rng(1000 + tile + len(sizes))
    n = 500
    recs, valid, ref_in = _synthetic_records(rng, len(sizes), n, sizes, tile)
    N = n * len(sizes)
    # view b sees Gaussians [b n, (b+1) n): ragged per-view ranges in one global array
    views = ViewSpec([w for w, _ in sizes], [h for _, h in sizes], [b * n for b in range(len(sizes))],
                     [(b + 1) * n for b in range(len(sizes))])
    keys, vals, ranges, counts, base = bin_reference(
        ref_in, [(w, h, b * n) for b, (w, h) in enumerate(sizes)], tile)
    n_cand = int(sum(int(c.sum()) for c in counts))
    cap = max(n_cand, 1)
    buf = r.buffers(views, N, 0, cap)
    r.bin_records(views, N, torch.from_numpy(recs).cuda(), torch.from_numpy(valid.astype(np.uint8)).cuda(), buf)
    torch.cuda.synchronize()
    sv = saved_arrays(buf, views)
    # K counts the candidate tiles; the ones the ellipse test drops leave the lists
    assert sv["K"] == n_cand and not sv["overflow"]
    assert np.array_equal(sv["pair_count"], np.concatenate(counts))
    kept = len(keys)
    assert kept <= n_cand and sv["n_listed"] == kept
    # pair ids -> Gaussian ids (view b's pairs start at pair_base[b] = b n and map to b n + local)
    gauss = sv["tile_pairs"]  # here pair id == Gaussian id because ranges are [b n, (b+1) n)
    # main gate, independent of the float32 decision steps: tile membership equals the float64
    # statement of the tile rule up to candidates within rounding of the level, and every
    # tile's list is in (float32 depth bits, Gaussian index) order
    f64_kept, f64_amb = membership_f64(ref_in, [(w, h, b * n) for b, (w, h) in enumerate(sizes)], tile)
    zbits = recs[:, 6].view(np.uint32).astype(np.int64)
    got = set()
    for t, (s0, s1) in enumerate(sv["ranges"]):
        lst = gauss[s0:s1]
        got |= {(t, int(g)) for g in lst}
        order = sorted(lst.tolist(), key=lambda g: (zbits[g], g))
        assert lst.tolist() == order, t
    assert len(got) == sv["n_listed"]
    assert got - f64_amb == f64_kept
    # and bit for bit with the float32 steps of the rule (the definition the kernel evaluates)
    assert np.array_equal(gauss, vals.astype(np.int64))
    zb = recs[:, 6].view(np.uint32).astype(np.uint64)[gauss]
    gkeys = (sv["tile_keys"].astype(np.uint64) << np.uint64(32)) | zb
    assert np.array_equal(gkeys, keys)
    assert np.array_equal(sv["ranges"], ranges.astype(np.int64))
    _check_work_list(sv["work"], sv["ranges"])


def test_binning_bit_exact_with_long_tile_lists():
    """Two views of one and six tiles, each seen by 14,000 Gaussians: lists of thousands of
    entries (over 10,000 in one tile) in the order (float32 depth bits, then pair id; the
    quantised depths tie often)."""
    from paper_2510_26358_amd.rasterizer import Rasterizer, ViewSpec
    r = Rasterizer(0, tile=16, batch=256, px_per_thread=1)
    rng = np.random.default_rng(1099)
    n, sizes = 14_000, [(16, 16), (40, 20)]
    recs, valid, ref_in = _synthetic_records(rng, len(sizes), n, sizes, 16, margin=0)
    N = n * len(sizes)
    views = ViewSpec([w for w, _ in sizes], [h for _, h in sizes], [0, n], [n, 2 * n])
    keys, vals, ranges, counts, base = bin_reference(ref_in, [(w, h, b * n) for b, (w, h) in enumerate(sizes)], 16)
    lengths = ranges[:, 1] - ranges[:, 0]
    assert lengths.max() > 8192
    cap = int(sum(int(c.sum()) for c in counts))
    buf = r.buffers(views, N, 0, cap)
    r.bin_records(views, N, torch.from_numpy(recs).cuda(), torch.from_numpy(valid.astype(np.uint8)).cuda(), buf)
    torch.cuda.synchronize()
    sv = saved_arrays(buf, views)
    assert sv["K"] == cap and sv["n_listed"] == len(keys)
    assert np.array_equal(sv["tile_pairs"], vals.astype(np.int64))
    assert np.array_equal(sv["ranges"], ranges.astype(np.int64))
    _check_work_list(sv["work"], sv["ranges"])


@pytest.mark.parametrize("keep_frac", [0.2, 0.6, 0.97])
def test_binning_bit_exact_with_several_sort_tiles_per_workgroup(keep_frac):
    """120,000 pairs in one 320 x 240 view: each radix workgroup of the depth sort owns four
    2,048-item tiles, so its dropping first pass packs the kept pairs of several tiles before
    ranking them (a fifth valid: one ranking round for all four; 60 %: rounds across tile
    boundaries; 97 %: about one per tile), and the tile sort's workgroups own several tiles
    too; lists, keys and ranges bit for bit against the reference."""
    from paper_2510_26358_amd.rasterizer import Rasterizer, ViewSpec
    r = Rasterizer(0, tile=16, batch=256, px_per_thread=1)
    rng = np.random.default_rng(1200 + int(100 * keep_frac))
    n, sizes = 120_000, [(320, 240)]
    recs, valid, ref_in = _synthetic_records(rng, 1, n, sizes, 16, keep_frac=keep_frac)
    views = ViewSpec([320], [240], [0], [n])
    keys, vals, ranges, counts, base = bin_reference(ref_in, [(320, 240, 0)], 16)
    cap = int(sum(int(c.sum()) for c in counts))
    buf = r.buffers(views, n, 0, cap)
    r.bin_records(views, n, torch.from_numpy(recs).cuda(), torch.from_numpy(valid.astype(np.uint8)).cuda(), buf)
    torch.cuda.synchronize()
    sv = saved_arrays(buf, views)
    assert sv["K"] == cap and not sv["overflow"] and sv["n_listed"] == len(keys)
    assert np.array_equal(sv["pair_count"], np.concatenate(counts))
    assert np.array_equal(sv["tile_pairs"], vals.astype(np.int64))
    zb = recs[:, 6].view(np.uint32).astype(np.uint64)[sv["tile_pairs"]]
    assert np.array_equal((sv["tile_keys"].astype(np.uint64) << np.uint64(32)) | zb, keys)
    assert np.array_equal(sv["ranges"], ranges.astype(np.int64))
    _check_work_list(sv["work"], sv["ranges"])


def _check_work_list(work, ranges):
    """The raster work list: every tile exactly once; strips of 8 consecutive tiles dealt
    round-robin to 8 interleaved lists (workgroup g in list g % 8); each list by descending
    4 log2(length + 1) bucket (a float32 bucket boundary may differ from the float64 one by
    rounding, so pairs within 1e-4 of an integer are not held to it); padding only at the
    ends of the lists."""
    NO = 0xFFFFFFFF
    n_t = len(ranges)
    strips = -(-n_t // 8)
    assert len(work) == 8 * (-(-strips // 8)) * 8
    assert sorted(work[work != NO].tolist()) == list(range(n_t))
    level = 4 * np.log2((ranges[:, 1] - ranges[:, 0]).astype(np.float64) + 1)
    for x in range(8):
        lst = work[x::8]
        real = lst[lst != NO]
        assert np.all(lst[len(real):] == NO)  # padding is a suffix
        assert np.all((real // 8) % 8 == x)
        lv = level[real]
        b = np.minimum(63, np.floor(lv))
        up = np.nonzero(b[1:] > b[:-1])[0]
        near = np.abs(lv - np.round(lv)) < 1e-4
        assert all(near[i] or near[i + 1] for i in up), (x, up[:5])


def test_misaligned_buffers_are_rejected_before_any_launch():
    """The kernels read records and sorted keys as 16-byte vectors: buffers that do not start
    on a 16-byte boundary are refused on the host, and an aligned call still works."""
    import ctypes as C
    from paper_2510_26358_amd import _lib as L
    from paper_2510_26358_amd.rasterizer import Rasterizer, ViewSpec, _stream
    r = Rasterizer(0, tile=16, batch=256, px_per_thread=1)
    rng = np.random.default_rng(77)
    recs, valid, _ = _synthetic_records(rng, 1, 64, [(64, 48)], 16)
    views = ViewSpec([64], [48], [0], [64])
    buf = r.buffers(views, 64, 0, 4096)
    rec_t = torch.from_numpy(recs).cuda()
    val_t = torch.from_numpy(valid.astype(np.uint8)).cuda()
    raw = torch.zeros(recs.size + 4, dtype=torch.float32, device="cuda")
    shifted = raw[1:1 + recs.size]            # 4 bytes past an aligned start
    shifted.copy_(rec_t.reshape(-1))

    def call(records, saved, ws):
        return r.lib.ags_bin_records(r.ctx, C.byref(views.c), 64, records, val_t.data_ptr(), buf.capacity,
                                     saved, ws, buf.sizes.fwd_ws_bytes, _stream())
    saved, ws = buf.saved.data_ptr(), buf.fwd_ws.data_ptr()
    assert call(shifted.data_ptr(), saved, ws) == L.AGS_ERR_INVALID_ARG
    assert call(rec_t.data_ptr(), saved + 8, ws) == L.AGS_ERR_INVALID_ARG
    assert call(rec_t.data_ptr(), saved, ws + 4) == L.AGS_ERR_INVALID_ARG
    assert call(rec_t.data_ptr(), saved, ws) == L.AGS_OK
    torch.cuda.synchronize()


def test_overflow_is_flagged_and_recovered(ras):
    sc = scenes.tiny_scene()
    from paper_2510_26358_amd.rasterizer import SplatParams, ViewSpec, cameras_tensor
    views = ViewSpec.from_scene(sc)
    p = SplatParams.from_scene(sc)
    cams = cameras_tensor(sc.cameras)
    buf = ras.buffers(views, p.n, p.sh_degree, 64)
    out = ras.outputs(views)
    ras.forward_into(p, cams, views, buf, out)
    k, v, over, keff = buf.counters()
    assert over == 1 and keff == 64 and k > 64
    out2, buf2 = ras.render(p, cams, views, capacity=64)
    assert buf2.counters()[2] == 0 and buf2.capacity >= k
    ref, _ = run_forward(sc, ras, capacity=int(k))
    assert np.array_equal(out2[0].cpu().numpy(), np.concatenate([r["rgb"].reshape(-1) for r in ref]))


def test_loss_and_gradients_tiny_l1(ras):
    sc = scenes.tiny_scene()
    g = run_loss_backward(sc, ras)
    ref = loss_and_grads(sc, RenderSettings())
    print("loss", g["loss"], ref["loss"], "excluded gaussians", ref["amb_gauss"].sum())
    assert abs(g["loss"] - ref["loss"]) <= 1e-5 * max(1, abs(ref["loss"]))
    for name in ["means", "log_scales", "quats", "opacity_logits", "sh"]:
        ok, msg = grad_close(g["grads"][name], ref["grads"][name], ref["amb_gauss"])
        print(name, msg)
        assert ok, (name, msg)
    ok, msg = grad_close(g["pose"], ref["pose"])
    print("pose", msg)
    assert ok, msg


@pytest.mark.parametrize("alpha_min", [1e-3, 2e-2])
def test_forward_and_gradients_with_another_alpha_cutoff(alpha_min):
    """The configured alpha_min sets both the keep test and the footprint box the tile lists
    come from: with a cutoff below the default 1/255 the boxes grow (no contributing pair is
    left out of the lists), above it they shrink."""
    from paper_2510_26358_amd.rasterizer import Rasterizer
    r = Rasterizer(0, alpha_min=alpha_min)
    s = RenderSettings(alpha_min=alpha_min)
    sc = scenes.tiny_scene()
    gpu, _ = run_forward(sc, r)
    _compare_forward(gpu, render(sc, s), sc)
    g = run_loss_backward(sc, r)
    ref = loss_and_grads(sc, s)
    print("loss", g["loss"], ref["loss"], "excluded gaussians", ref["amb_gauss"].sum())
    assert abs(g["loss"] - ref["loss"]) <= 1e-5 * max(1, abs(ref["loss"]))
    for name in ["means", "log_scales", "quats", "opacity_logits", "sh"]:
        ok, msg = grad_close(g["grads"][name], ref["grads"][name], ref["amb_gauss"])
        print(name, msg)
        assert ok, (name, msg)
    ok, msg = grad_close(g["pose"], ref["pose"])
    print("pose", msg)
    assert ok, msg


@pytest.mark.parametrize("seed,n_views", [(201, 1), (202, 2)])
def test_loss_and_gradients_sh3_lidar(ras, seed, n_views):
    sc = random_scene(seed, n=400, sh_degree=3, n_views=n_views, width=64, height=48, f=60.0)
    g = run_loss_backward(sc, ras, w_l1=0.8, lam=0.5)
    ref = loss_and_grads(sc, RenderSettings(), w_l1=0.8, lam=0.5)
    print("loss", g["loss"], ref["loss"], "excluded", ref["amb_gauss"].sum())
    assert abs(g["loss"] - ref["loss"]) <= 1e-5 * max(1, abs(ref["loss"]))
    for name in ["means", "log_scales", "quats", "opacity_logits", "sh"]:
        ok, msg = grad_close(g["grads"][name], ref["grads"][name], ref["amb_gauss"])
        print(name, msg)
        assert ok, (name, msg)
    ok, msg = grad_close(g["pose"], ref["pose"])
    print("pose", msg)
    assert ok, msg


# Every (tile, LDS batch, pixels per thread) launch shape the library accepts, each used for
# both passes, and three forward/backward pairs of different shapes on one tile size: the
# benchmark's autotuner may pick any of them (backward batches of 64 records with two waves
# merge the waves' sums in LDS; the others add them per wave).  Two 70x45 views (ragged tiles for 8, 16 and 32),
# up to ~90 contributors per pixel, so the 64- and 128-record batches loop.
_SHAPES = [(8, 64, 1), (8, 128, 1), (16, 128, 1), (16, 256, 1), (16, 64, 2), (16, 128, 2), (16, 256, 2),
           (16, 64, 4), (32, 256, 4), (32, 512, 2)]
_SHAPE_CASES = [(s, s[1:]) for s in _SHAPES] + [((16, 256, 1), (128, 2)), ((16, 256, 1), (64, 2)),
                                                ((16, 64, 4), (256, 1))]
_shape_ref = {}


def _shape_reference():
    if not _shape_ref:
        sc = random_scene(233, n=900, sh_degree=3, n_views=2, width=70, height=45, f=55.0)
        _shape_ref.update(scene=sc, fwd=render(sc, RenderSettings()),
                          loss=loss_and_grads(sc, RenderSettings(), w_l1=0.8, lam=0.5))
    return _shape_ref


@pytest.mark.parametrize("fwd,bwd", _SHAPE_CASES, ids=[f"fwd{f}-bwd{b}" for f, b in _SHAPE_CASES])
def test_every_launch_shape_matches_the_oracle(fwd, bwd):
    from paper_2510_26358_amd.rasterizer import Rasterizer
    ref = _shape_reference()
    sc, lr = ref["scene"], ref["loss"]
    r = Rasterizer(0, tile=fwd[0], batch=fwd[1], px_per_thread=fwd[2], batch_bwd=bwd[0], px_per_thread_bwd=bwd[1])
    print("forward", fwd, "backward", bwd, flush=True)
    g = run_loss_backward(sc, r, w_l1=0.8, lam=0.5)
    _compare_forward(g["fwd"], ref["fwd"], sc)
    print("loss", g["loss"], lr["loss"], "excluded", lr["amb_gauss"].sum())
    assert abs(g["loss"] - lr["loss"]) <= 1e-5 * max(1, abs(lr["loss"]))
    for name in ["means", "log_scales", "quats", "opacity_logits", "sh"]:
        ok, msg = grad_close(g["grads"][name], lr["grads"][name], lr["amb_gauss"])
        print(name, msg)
        assert ok, (name, msg)
    ok, msg = grad_close(g["pose"], lr["pose"])
    print("pose", msg)
    assert ok, msg


def test_check_finite_counts_non_finite_parameters(ras):
    from paper_2510_26358_amd.rasterizer import SplatParams
    p = SplatParams.from_scene(scenes.tiny_scene())
    assert ras.check_finite(p) == 0
    q = p.clone()
    q.means[1, 5] = float("nan")
    q.quats[3, 7] = float("inf")
    q.sh[0, 2, 11] = float("-inf")
    q.opacity_logits[p.n - 1] = float("nan")
    assert ras.check_finite(q) == 4


def _many_view_scene(seed, n_views, n=300):
    """The largest view count the ABI accepts, with ragged image sizes and per-view Gaussian
    ranges (some views see every Gaussian, others a slice), each camera slightly rotated
    and shifted; random targets and a few LiDAR pixels per view."""
    import math
    from tests.oracle_helpers import camera
    sc = random_scene(seed, n=n, sh_degree=2, n_views=1, width=24, height=16, f=22.0)
    rng = np.random.default_rng(seed + 1)
    cams, gts, lidar = [], [], []
    for b in range(n_views):
        ay, ax = rng.uniform(-0.15, 0.15), rng.uniform(-0.1, 0.1)
        Ry = np.array([[math.cos(ay), 0, math.sin(ay)], [0, 1, 0], [-math.sin(ay), 0, math.cos(ay)]])
        Rx = np.array([[1, 0, 0], [0, math.cos(ax), -math.sin(ax)], [0, math.sin(ax), math.cos(ax)]])
        w, h = 16 + 8 * (b % 3), 12 + 4 * (b % 2)
        c = camera(R=Rx @ Ry, t=rng.uniform(-0.2, 0.2, 3), f=18.0 + b % 4, width=w, height=h)
        if b % 4 == 3:
            c.g_begin, c.g_end = n // 4, 3 * n // 4
        else:
            c.g_begin, c.g_end = 0, n
        cams.append(c)
        gts.append(rng.uniform(0, 1, (3, h, w)))
        m = 6
        pix = np.sort(rng.choice(w * h, m, replace=False)).astype(np.int32)
        lidar.append({"pix": pix, "depth": rng.uniform(2.5, 3.5, m), "sigma": rng.uniform(0.5, 1.0, m)})
    sc.cameras, sc.gt_rgb, sc.lidar = cams, gts, lidar
    return sc


def test_loss_and_gradients_at_the_maximum_view_count(ras):
    from paper_2510_26358_amd._lib import AGS_MAX_VIEWS
    sc = _many_view_scene(211, AGS_MAX_VIEWS)
    g = run_loss_backward(sc, ras, w_l1=0.7, lam=0.5)
    ref = loss_and_grads(sc, RenderSettings(), w_l1=0.7, lam=0.5)
    print("views", len(sc.cameras), "loss", g["loss"], ref["loss"], "excluded", ref["amb_gauss"].sum())
    assert abs(g["loss"] - ref["loss"]) <= 1e-5 * max(1, abs(ref["loss"]))
    for name in ["means", "log_scales", "quats", "opacity_logits", "sh"]:
        ok, msg = grad_close(g["grads"][name], ref["grads"][name], ref["amb_gauss"])
        print(name, msg)
        assert ok, (name, msg)
    ok, msg = grad_close(g["pose"], ref["pose"])
    print("pose", msg)
    assert ok, msg
