"""Graph-captured refinement step (forward, fused-loss backward, Adam, se(3) pose update) and
the pose-gradient check of the refinement workload: on a 4k-Gaussian crop of the 2M-Gaussian
map, the HIP pose gradient against FP64 central finite differences (step 1e-6) of the
oracle, every 10 steps of the loop."""
import numpy as np
import pytest
import torch

from oracle.render import frozen_objective, loss_and_grads
from oracle.settings import RenderSettings
from paper_2510_26358_amd import scenes
from paper_2510_26358_amd.rasterizer import (LossTargets, Rasterizer, SplatParams, ViewSpec,
                                             cameras_tensor)
from paper_2510_26358_amd.refine import Refiner
from paper_2510_26358_amd.scenes import Camera, Scene
from tests.oracle_helpers import random_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ras():
    return Rasterizer(0)


def _refiner(ras, sc, capacity=None, fused_adam=True):
    views = ViewSpec.from_scene(sc)
    p = SplatParams.from_scene(sc)
    cams = cameras_tensor(sc.cameras)
    tg = LossTargets.from_scene(sc, views, lambda_lidar=0.5)
    return Refiner(ras, p, cams, views, tg, capacity=capacity, fused_adam=fused_adam)


@pytest.mark.parametrize("fused_adam", [True, False])
def test_graph_replay_matches_eager_steps(ras, fused_adam):
    sc = random_scene(401, n=3000, sh_degree=3, n_views=2, width=96, height=72, f=80.0)
    a = _refiner(ras, sc, fused_adam=fused_adam)
    b = _refiner(ras, sc, capacity=a.buf.capacity, fused_adam=fused_adam)
    b.capture()
    losses = []
    for it in range(4):
        a.step()
        b.replay()
        # unrelated eager work and a synchronisation between replays
        torch.ones(1000, device="cuda").sum().item()
        torch.cuda.synchronize()
        assert a.check_capacity() and b.check_capacity()
        for x, y in zip(a.p.tensors(), b.p.tensors()):
            assert torch.allclose(x, y, rtol=1e-5, atol=1e-6), it
        assert torch.allclose(a.cams, b.cams, rtol=1e-5, atol=1e-6)
        assert int(a.step_no.item()) == int(b.step_no.item()) == it + 2
        losses.append(a.loss.item())
        assert abs(a.loss.item() - b.loss.item()) <= 1e-4 * abs(a.loss.item())
    assert losses[-1] < losses[0]


@pytest.mark.parametrize("deg", [3, 1, 0])
def test_fused_backward_adam_equals_backward_then_adam(ras, deg):
    """ags_render_bwd_adam against ags_render_bwd followed by ags_adam_step over four steps
    (moments non-zero after the first, bias corrections changing): parameters, both Adam
    moments, the pose gradient, the poses and the loss agree to the tolerance of the graph
    replay test.  Not bit for bit: the per-pair adjoint sums of the raster backward are float
    atomics, whose order differs from run to run, so two backward passes differ in the last
    bits of their gradients."""
    sc = random_scene(411 + deg, n=1500, sh_degree=deg, n_views=2, width=80, height=60, f=70.0)
    a = _refiner(ras, sc, fused_adam=True)
    b = _refiner(ras, sc, capacity=a.buf.capacity, fused_adam=False)
    for it in range(4):
        a.step()
        b.step()
        torch.cuda.synchronize()
        assert a.check_capacity() and b.check_capacity()
        for name, x, y in zip(("p", "m", "v"), (a.p, a.m, a.v), (b.p, b.m, b.v)):
            for fx, fy in zip(x.tensors(), y.tensors()):
                tol = 1e-6 if name == "p" else 1e-6 * max(fy.abs().max().item(), 1e-30)
                assert torch.allclose(fx, fy, rtol=1e-5, atol=tol), (it, name, (fx - fy).abs().max().item())
        assert torch.allclose(a.pose_grad, b.pose_grad, rtol=1e-4, atol=1e-6 * b.pose_grad.abs().max().item()), it
        assert torch.allclose(a.cams, b.cams, rtol=1e-5, atol=1e-6), it
        assert abs(a.loss.item() - b.loss.item()) <= 1e-5 * abs(b.loss.item()), it


def test_fused_backward_adam_arguments(ras):
    """The fused call leaves grads.sh alone (it may be NULL) and refuses accumulation; both
    checked on the host before any launch."""
    import ctypes as C
    from paper_2510_26358_amd import _lib as L
    from paper_2510_26358_amd.rasterizer import _fwd_out, _ptr, _stream
    sc = random_scene(431, n=300, sh_degree=3, n_views=1, width=48, height=32, f=50.0)
    r = _refiner(ras, sc)
    ras.forward_into(r.p, r.cams, r.views, r.buf, r.out)
    fo, g, mc, vc, lc = _fwd_out(r.out), r.p.c(), r.m.c(), r.v.c(), r.targets.c()

    def call(sh_ptr, acc):
        ptrs = [t.data_ptr() for t in r.grads.tensors()]
        gr = L.Grads(ptrs[0], ptrs[1], ptrs[2], ptrs[3], sh_ptr, r.pose_grad.data_ptr(), acc, None, None)
        return ras.lib.ags_render_bwd_adam(ras.ctx, C.byref(r.views.c), C.byref(g), _ptr(r.cams), r.buf.capacity,
                                           C.byref(fo), _ptr(r.buf.saved), None, C.byref(lc), C.byref(gr),
                                           _ptr(r.loss), C.byref(r.hp), C.byref(mc), C.byref(vc), _ptr(r.step_no),
                                           _ptr(r.buf.bwd_ws), r.buf.sizes.bwd_ws_bytes, _stream())
    assert call(r.grads.sh.data_ptr(), 1) == L.AGS_ERR_INVALID_ARG
    r.grads.sh.fill_(7.0)
    assert call(r.grads.sh.data_ptr(), 0) == L.AGS_OK
    assert call(None, 0) == L.AGS_OK
    torch.cuda.synchronize()
    assert torch.equal(r.grads.sh, torch.full_like(r.grads.sh, 7.0))
    assert torch.isfinite(r.p.sh).all() and int(r.step_no.item()) == 1


def _crop(sc, cams_np, params_aos, rng, n_keep=4096, win=128):
    """4096 Gaussians nearest (in 3D, in front of the camera) to the ray through the centre
    of a seeded 128x128 window of view 0, seen through a window camera whose principal
    point is shifted to the window."""
    cam0 = sc.cameras[0]
    R = cams_np[0, :9].reshape(3, 3).astype(np.float64)
    t = cams_np[0, 9:12].astype(np.float64)
    x0 = int(rng.integers(0, cam0.width - win))
    y0 = int(rng.integers(0, cam0.height - win))
    ray = np.array([(x0 + win / 2 - cam0.cx) / cam0.fx, (y0 + win / 2 - cam0.cy) / cam0.fy, 1.0])
    ray /= np.linalg.norm(ray)
    means, ls, q, lo, sh = params_aos
    xc = means.astype(np.float64) @ R.T + t
    along = xc @ ray
    dist = np.linalg.norm(xc - along[:, None] * ray[None, :], axis=1)
    dist[along < 0.5] = np.inf
    keep = np.sort(np.argsort(dist)[:n_keep])
    cam = Camera(R.astype(np.float32), t.astype(np.float32), cam0.fx, cam0.fy, cam0.cx - x0, cam0.cy - y0,
                 win, win, 0, len(keep))
    gt = sc.gt_rgb[0][:, y0:y0 + win, x0:x0 + win].copy()
    lid = sc.lidar[0]
    px, py = lid["pix"] % cam0.width, lid["pix"] // cam0.width
    inside = (px >= x0) & (px < x0 + win) & (py >= y0) & (py < y0 + win)
    lidar = {"pix": ((py[inside] - y0) * win + (px[inside] - x0)).astype(np.int32),
             "depth": lid["depth"][inside], "sigma": lid["sigma"][inside]}
    return Scene(means[keep].copy(), ls[keep].copy(), q[keep].copy(), lo[keep].copy(), sh[keep].copy(),
                 sc.sh_degree, [cam], [gt], [lidar], name="crop")


def test_refinement_pose_gradient_matches_fp64_finite_differences_every_10_steps(ras):
    """The captured refinement loop (2M Gaussians, 4 views) run for 50 Adam iterations; at
    steps 0, 10, ..., 50 the pose gradient of a 4,096-Gaussian crop of the current state is
    checked against FP64 central finite differences (h = 1e-6, decisions frozen).  Both sides
    differentiate the loss over the crop's pixels whose decisions float32 rounding cannot
    flip (pixels the oracle flags as ambiguous, and their LiDAR targets, are left out of the
    objective on both sides)."""
    sc = scenes.refinement_scene()
    st = scenes.perturb(sc, seed=77)
    views = ViewSpec.from_scene(st)
    p = SplatParams.from_scene(st)
    cams = cameras_tensor(st.cameras)
    tg = LossTargets.from_scene(sc, views, lambda_lidar=0.1)
    ref = Refiner(ras, p, cams, views, tg)
    ref.capture()
    rng = np.random.default_rng(2515)
    s = RenderSettings()
    for it in range(51):
        if it % 10 == 0:
            torch.cuda.synchronize()
            crop = _crop(sc, ref.cams.cpu().numpy(), ref.p.to_numpy_aos(), rng)
            flags = loss_and_grads(crop, s, lam=0.1)["views"][0]
            keep = np.asarray(flags["pix"])[~flags["ambiguous"]]
            lid = crop.lidar[0]
            inside = np.isin(lid["pix"], keep)
            crop.lidar = [{k: np.asarray(v)[inside] for k, v in lid.items()}]
            cv = ViewSpec.from_scene(crop)
            cp = SplatParams.from_scene(crop)
            cc = cameras_tensor(crop.cameras)
            ct = LossTargets.from_scene(crop, cv, masks=[keep], lambda_lidar=0.1)
            out, buf = ras.render(cp, cc, cv)
            gr = cp.zeros_like()
            pose = torch.zeros(1, 6, device="cuda")
            ras.backward_into(cp, cc, cv, buf, out, gr, pose, loss=ct)
            torch.cuda.synchronize()
            g_gpu = pose.cpu().numpy()[0].astype(np.float64)
            r = loss_and_grads(crop, s, masks=[keep], lam=0.1)
            h = 1e-6
            fd = np.zeros(6)
            for j in range(6):
                d = np.zeros((1, 6))
                d[0, j] = h
                fd[j] = (frozen_objective(crop, r["decisions"], s, masks=[keep], lam=0.1, deltas=d) -
                         frozen_objective(crop, r["decisions"], s, masks=[keep], lam=0.1, deltas=-d)) / (2 * h)
            print(f"step {it}: {int(flags['ambiguous'].sum())} ambiguous pixels left out")
            # each component is a float32 sum over every pixel and Gaussian of the crop; as the
            # loop converges one component can nearly cancel while its terms stay as large as
            # the others, so components are held to 1e-3 of the largest one and the vector to
            # 1e-3 in norm
            err = np.abs(g_gpu - fd)
            scale = np.abs(fd).max()
            print(f"step {it}: gpu {np.array2string(g_gpu, precision=5)} fd {np.array2string(fd, precision=5)} "
                  f"max err / max |fd| {np.max(err) / scale:.2e}")
            assert np.linalg.norm(g_gpu - fd) <= 1e-3 * np.linalg.norm(fd)
            assert np.all(err <= 1e-3 * scale)
        if it < 50:
            ref.replay()
    assert ref.check_capacity()


def test_checkpoint_resume_continues_the_loop(ras, tmp_path):
    """Three steps, save, three more; a fresh loop loaded from the checkpoint and run for
    three steps lands on the same state (float atomics leave last-bit differences in the
    gradients, so parameters agree to rounding, the step counter exactly)."""
    sc = random_scene(402, n=2000, sh_degree=2, n_views=2, width=80, height=60, f=70.0)
    a = _refiner(ras, sc)
    for _ in range(3):
        a.step()
    path = str(tmp_path / "ckpt.npz")
    a.save(path)
    for _ in range(3):
        a.step()
    b = _refiner(ras, sc, capacity=a.buf.capacity)
    b.load(path)
    for _ in range(3):
        b.step()
    sa, sb = a.state(), b.state()
    assert int(sa["step"][0]) == int(sb["step"][0]) == 7
    for k in sa:
        if k in ("step", "sh_degree"):
            continue
        assert np.allclose(sa[k], sb[k], rtol=1e-4, atol=1e-6), k
    # a checkpoint of another shape is refused
    other = random_scene(403, n=100, sh_degree=2, n_views=2, width=80, height=60, f=70.0)
    c = _refiner(ras, other)
    with pytest.raises(ValueError):
        c.load(path)
