"""ags_lifecycle_step_noalloc (scratch in the library's static device array, for callers that
cannot allocate) against ags_lifecycle_step (caller workspace): identical outputs on two calls
in a row, the second on a smaller input, plus the host-side size refusal."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2510_26358_amd import _lib as L
from paper_2510_26358_amd.rasterizer import LifecycleParams, Rasterizer, SplatParams
from tests.test_gpu_lifecycle import _lifecycle_inputs, _to_gpu

pytestmark = pytest.mark.gpu


def _call(ras, lp, inputs, sh_degree, noalloc):
    params, m, v, accum, count, noise = inputs
    p, pm, pv = _to_gpu(params, sh_degree), _to_gpu(m, sh_degree), _to_gpu(v, sh_degree)
    n = p.n
    outs = [SplatParams.empty(2 * n, sh_degree) for _ in range(3)]
    for o in outs:
        for t in o.tensors():
            t.fill_(-7.0)  # rows beyond n_out must stay untouched by both calls
    n_out = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    actions = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    sg, sc = torch.from_numpy(accum).cuda(), torch.from_numpy(count).cuda()
    nz = torch.from_numpy(noise).cuda()
    gi, mi, vi = p.c(), pm.c(), pv.c()
    go, mo, vo = [o.c() for o in outs]
    lc = lp.c()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [ras.ctx, C.byref(lc), C.byref(gi), C.byref(mi), C.byref(vi), C.c_void_p(sg.data_ptr()),
            C.c_void_p(sc.data_ptr()), C.c_void_p(nz.data_ptr()), C.byref(go), C.byref(mo), C.byref(vo),
            C.c_void_p(n_out.data_ptr()), C.c_void_p(actions.data_ptr())]
    if noalloc:
        rc = ras.lib.ags_lifecycle_step_noalloc(*args, stream)
    else:
        ws = torch.empty(max(ras.lifecycle_workspace(n), 1), dtype=torch.uint8, device="cuda")
        rc = ras.lib.ags_lifecycle_step(*args, C.c_void_p(ws.data_ptr()), ws.numel(), stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return int(n_out.item()), actions.cpu().numpy(), [[t.cpu() for t in o.tensors()] for o in outs]


@pytest.mark.parametrize("n,sh_degree,seed", [(300_000, 3, 901), (40_000, 1, 902)])
def test_noalloc_lifecycle_equals_workspace_lifecycle(n, sh_degree, seed):
    ras = Rasterizer(0)
    lp = LifecycleParams(do_prune=True, do_densify=True, do_reset=True)
    inputs = _lifecycle_inputs(seed, n, sh_degree, lp)
    # the no-alloc call first and last, so a stale array from the larger call would show
    a = _call(ras, lp, inputs, sh_degree, noalloc=True)
    b = _call(ras, lp, inputs, sh_degree, noalloc=False)
    print(f"n {n}: n_out {a[0]}, actions {np.bincount(a[1], minlength=4)}")
    assert a[0] == b[0] and 0 < a[0] <= 2 * n
    assert np.array_equal(a[1], b[1])
    for oa, ob in zip(a[2], b[2]):
        for ta, tb in zip(oa, ob):
            assert torch.equal(ta, tb)


def test_two_noalloc_calls_in_a_row_the_second_smaller():
    ras = Rasterizer(0)
    lp = LifecycleParams(do_prune=True, do_densify=True, do_reset=False)
    big = _lifecycle_inputs(911, 500_000, 2, lp)
    small = _lifecycle_inputs(912, 3_000, 2, lp)
    ra = _call(ras, lp, big, 2, noalloc=True)
    rb = _call(ras, lp, small, 2, noalloc=True)
    ea = _call(ras, lp, big, 2, noalloc=False)
    eb = _call(ras, lp, small, 2, noalloc=False)
    for got, exp in [(ra, ea), (rb, eb)]:
        assert got[0] == exp[0]
        assert np.array_equal(got[1], exp[1])
        for oa, ob in zip(got[2], exp[2]):
            for ta, tb in zip(oa, ob):
                assert torch.equal(ta, tb)


def test_noalloc_refuses_inputs_above_its_maximum():
    ras = Rasterizer(0)
    lp = LifecycleParams()
    p = SplatParams.empty(4, 0)
    g = p.c()
    g.n = L.LIFECYCLE_NOALLOC_MAX_N + 1  # refused on the host before any device access
    lc = lp.c()
    z = C.c_void_p(p.means.data_ptr())
    rc = ras.lib.ags_lifecycle_step_noalloc(ras.ctx, C.byref(lc), C.byref(g), C.byref(g), C.byref(g), z, z, z,
                                            C.byref(g), C.byref(g), C.byref(g), z, None, C.c_void_p(0))
    assert rc == L.AGS_ERR_WORKSPACE
