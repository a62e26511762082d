"""The C ABI's own behaviour on the GPU: the autotuner entry point, workspace refusals and
LiDAR targets outside their view."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle.render import loss_and_grads
from oracle.settings import RenderSettings
from paper_2510_26358_amd import _lib as L
from paper_2510_26358_amd.rasterizer import (LossTargets, Rasterizer, SplatParams, ViewSpec,
                                             cameras_tensor)
from tests.gpu_helpers import run_loss_backward
from tests.oracle_helpers import random_scene

pytestmark = pytest.mark.gpu

SUPPORTED = {(8, 64, 1), (8, 128, 1), (16, 128, 1), (16, 256, 1), (16, 64, 2), (16, 128, 2), (16, 256, 2),
             (16, 64, 4), (32, 256, 4), (32, 512, 2)}


def _inputs(seed=501):
    sc = random_scene(seed, n=400, sh_degree=1, n_views=2, width=72, height=50, f=60.0)
    views = ViewSpec.from_scene(sc)
    return sc, views, SplatParams.from_scene(sc), cameras_tensor(sc.cameras), LossTargets.from_scene(sc, views)


def test_tune_times_every_compiled_shape_and_sets_a_supported_pick():
    sc, views, p, cams, tg = _inputs()
    ras = Rasterizer(0)
    ras.profile(True)
    from paper_2510_26358_amd.tune import tune
    res = tune(ras, p, cams, views, tg, steps=2, warmup=1, use_cache=False)
    best = res["best"]
    assert len(res["ms"]) == len(SUPPORTED)
    assert {(int(k.split("_")[0][1:]), int(k.split("_")[1][1:]), int(k.split("_")[2][1:])) for k in res["ms"]} \
        == SUPPORTED
    assert (best["tile"], best["batch"], best["ppt"]) in SUPPORTED
    assert (best["tile"], best["batch_bwd"], best["ppt_bwd"]) in SUPPORTED
    for e in res["ms"].values():
        assert e["step_ms"] > 0 and e["raster_fwd"] > 0 and e["raster_bwd"] > 0 and e["K"] > 0
    # the pick is set on the context: a step with it still matches the oracle
    assert (ras.cfg.tile, ras.cfg.batch, ras.cfg.px_per_thread) == (best["tile"], best["batch"], best["ppt"])
    g = run_loss_backward(sc, ras)
    ref = loss_and_grads(sc, RenderSettings())
    assert abs(g["loss"] - ref["loss"]) <= 1e-4 * max(1.0, abs(ref["loss"]))
    # the caller's profile is kept (the tuner's own timings do not leak into it)
    prof = ras.profile_read()
    assert prof["raster_fwd"][1] == 1 and prof["raster_bwd"][1] == 1


def test_too_small_workspaces_are_refused_before_any_launch():
    sc, views, p, cams, tg = _inputs(502)
    ras = Rasterizer(0)
    out, buf = ras.render(p, cams, views)
    torch.cuda.synchronize()
    s = buf.sizes
    # the context-keyed query gives the sizes of the configuration-keyed one
    q = L.Sizes()
    assert ras.lib.ags_workspace_query(ras.ctx, C.byref(views.c), p.n, p.sh_degree, buf.capacity, C.byref(q)) == 0
    assert (q.saved_bytes, q.fwd_ws_bytes, q.bwd_ws_bytes) == (s.saved_bytes, s.fwd_ws_bytes, s.bwd_ws_bytes)
    g = p.c()
    fo = L.FwdOut(out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), None)
    null = C.c_void_p(0)
    rc = ras.lib.ags_render_fwd(ras.ctx, C.byref(views.c), C.byref(g), C.c_void_p(cams.data_ptr()), buf.capacity,
                                C.byref(fo), C.c_void_p(buf.saved.data_ptr()), C.c_void_p(buf.fwd_ws.data_ptr()),
                                s.fwd_ws_bytes - 1, null)
    assert rc == L.AGS_ERR_WORKSPACE
    grads = p.zeros_like()
    pose = torch.zeros(views.n_views, 6, device="cuda")
    gr = L.Grads(*[t.data_ptr() for t in grads.tensors()], pose.data_ptr(), 0, None, None)
    lc = tg.c()
    rc = ras.lib.ags_render_bwd(ras.ctx, C.byref(views.c), C.byref(g), C.c_void_p(cams.data_ptr()), buf.capacity,
                                C.byref(fo), C.c_void_p(buf.saved.data_ptr()), None, C.byref(lc), C.byref(gr), None,
                                C.c_void_p(buf.bwd_ws.data_ptr()), s.bwd_ws_bytes - 1, null)
    assert rc == L.AGS_ERR_WORKSPACE
    assert torch.all(grads.means == 0)  # nothing was launched
    lc_ws = ras.lifecycle_workspace(p.n)
    ws = torch.empty(lc_ws, dtype=torch.uint8, device="cuda")
    outs = [SplatParams.empty(2 * p.n, p.sh_degree) for _ in range(3)]
    n_out = torch.zeros(1, dtype=torch.int32, device="cuda")
    from paper_2510_26358_amd.rasterizer import LifecycleParams
    lp = LifecycleParams(do_densify=False).c()
    m, v = p.zeros_like(), p.zeros_like()
    go, mo, vo = [o.c() for o in outs]
    rc = ras.lib.ags_lifecycle_step(ras.ctx, C.byref(lp), C.byref(g), C.byref(m.c()), C.byref(v.c()), None, None,
                                    None, C.byref(go), C.byref(mo), C.byref(vo), C.c_void_p(n_out.data_ptr()), None,
                                    C.c_void_p(ws.data_ptr()), lc_ws - 1, null)
    assert rc == L.AGS_ERR_WORKSPACE


def test_lidar_target_outside_its_view_makes_the_loss_nan():
    """The device targets cannot be checked on the host without a synchronisation: a pixel
    outside its view gets no adjoint (no access outside the image) and poisons the loss."""
    sc, views, p, cams, tg = _inputs(503)
    ras = Rasterizer(0)
    out, buf = ras.render(p, cams, views)
    grads = p.zeros_like()
    pose = torch.zeros(views.n_views, 6, device="cuda")
    loss = torch.zeros(1, device="cuda")
    ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss)
    torch.cuda.synchronize()
    assert np.isfinite(loss.item())
    bad = tg.depth_pix.clone()
    bad[tg.depth_offsets[1]] = views.widths[1] * views.heights[1]  # one past view 1's last pixel
    tg.depth_pix = bad
    ras.backward_into(p, cams, views, buf, out, grads, pose, loss=tg, loss_out=loss)
    torch.cuda.synchronize()
    assert np.isnan(loss.item())
