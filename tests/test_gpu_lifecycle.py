"""GPU parity of the lifecycle path (Sec. III-B, "Gaussian Splats Lifecycle Operations"): the
densification statistic the backward accumulates (|dL/d(u, v)| summed over the views that see a
Gaussian, and the number of those views) and the prune / split / duplicate / reset step, against
the oracle.  Decisions are taken in float32 on both sides; inputs are kept a few ulps away from
every threshold so that a 1-ulp difference between two exponentials cannot flip one."""
import math

import numpy as np
import pytest
import torch

from oracle import lifecycle as olc
from oracle.render import loss_and_grads
from oracle.settings import RenderSettings
from paper_2510_26358_amd import scenes
from tests.gpu_helpers import grad_close, run_loss_backward
from tests.oracle_helpers import random_scene

pytestmark = pytest.mark.gpu

NAMES = ["means", "log_scales", "quats", "opacity_logits", "sh"]


@pytest.fixture(scope="module")
def ras():
    from paper_2510_26358_amd.rasterizer import Rasterizer
    return Rasterizer(0)


def _check_stats(g, ref):
    st, rs = g["stats"], ref["stats"]
    amb = rs["ambiguous"] | ref["amb_gauss"]
    print("seen", int((rs["count"] > 0).sum()), "ambiguous", int(amb.sum()))
    assert np.array_equal(st["count"][~amb], rs["count"][~amb].astype(np.float32))
    ok, msg = grad_close(st["grad_accum"], rs["grad_accum"], amb)
    print("grad_accum", msg)
    assert ok, msg


@pytest.mark.parametrize("seed,n_views,ssim_w", [(301, 1, 0.0), (302, 2, 0.2)])
def test_densification_statistic_matches_oracle(ras, seed, n_views, ssim_w):
    sc = random_scene(seed, n=500, sh_degree=1, n_views=n_views, width=64, height=48, f=60.0)
    g = run_loss_backward(sc, ras, w_l1=0.8, lam=0.5, ssim_w=ssim_w, stats=True)
    ref = loss_and_grads(sc, RenderSettings(), w_l1=0.8, lam=0.5, ssim_w=ssim_w, stats=True)
    _check_stats(g, ref)


def test_densification_statistic_on_a_full_size_sample(ras):
    sc = scenes.single_view_scene()
    rng = np.random.default_rng(3031)
    lid = sc.lidar[0]
    pick = np.sort(rng.choice(len(lid["pix"]), 200, replace=False))
    sc.lidar = [{k: np.asarray(v)[pick] for k, v in lid.items()}]
    pix = np.unique(np.asarray(sc.lidar[0]["pix"], np.int64))
    g = run_loss_backward(sc, ras, masks=[pix], w_l1=0.3, lam=1.0, stats=True)
    ref = loss_and_grads(sc, RenderSettings(), masks=[pix], w_l1=0.3, lam=1.0, stats=True)
    _check_stats(g, ref)


def _away(x, thresholds, rel=1e-5):
    """True where the float32 value x lies at least rel (relative) from every threshold."""
    ok = np.ones(x.shape, bool)
    for t in thresholds:
        ok &= np.abs(x.astype(np.float64) - t) > rel * abs(t)
    return ok


def _lifecycle_inputs(seed, n, sh_degree, lp):
    """Seeded parameters spanning every rule: opacities around tau_opa / tau_reset, sizes from
    below s_min to above s_max, hot and cool statistics, some never seen.  Values within 1e-5
    (relative) of a threshold are drawn again."""
    rng = np.random.default_rng(seed)
    k = (sh_degree + 1) ** 2

    def draw(m):
        size = np.exp(rng.uniform(math.log(2e-5), math.log(0.6), m))
        aniso = np.exp(-rng.uniform(0.0, 1.5, (m, 3)))
        aniso[np.arange(m), rng.integers(0, 3, m)] = 1.0
        ls = np.log(size[:, None] * aniso).astype(np.float32)
        o = np.exp(rng.uniform(math.log(1e-3), math.log(0.99), m))
        logits = np.log(o / (1 - o)).astype(np.float32)
        count = rng.integers(0, 5, m).astype(np.float32)
        accum = (rng.exponential(lp.grad_threshold, m) * count).astype(np.float32)
        return ls, logits, count, accum

    ls, logits, count, accum = draw(n)
    while True:
        o32 = np.float32(1) / (np.float32(1) + np.exp(-logits))
        s32 = np.exp(ls.max(axis=1))
        g32 = accum / np.maximum(count, np.float32(1))
        bad = ~(_away(o32, [lp.tau_opa, lp.tau_reset]) & _away(s32, [lp.s_min, lp.s_max, lp.kappa, 2 * lp.s_init])
                & _away(g32, [lp.grad_threshold]))
        if not bad.any():
            break
        idx = np.nonzero(bad)[0]
        ls[idx], logits[idx], count[idx], accum[idx] = draw(len(idx))
    params = {"means": rng.normal(0, 2, (n, 3)).astype(np.float32), "log_scales": ls,
              "quats": rng.normal(size=(n, 4)).astype(np.float32), "opacity_logits": logits,
              "sh": rng.normal(0, 0.5, (n, k, 3)).astype(np.float32)}
    m = {kk: rng.normal(size=a.shape).astype(np.float32) for kk, a in params.items()}
    v = {kk: rng.random(size=a.shape).astype(np.float32) for kk, a in params.items()}
    noise = rng.normal(size=(n, 2, 3)).astype(np.float32)
    return params, m, v, accum, count, noise


def _to_gpu(d, sh_degree):
    from paper_2510_26358_amd.rasterizer import SplatParams
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    return SplatParams(f(d["means"].T), f(d["log_scales"].T), f(d["quats"].T), f(d["opacity_logits"]),
                       f(np.transpose(d["sh"], (1, 2, 0))), sh_degree)


def _aos(p):
    return dict(zip(NAMES, [a.astype(np.float64) for a in p.to_numpy_aos()]))


def _run_lifecycle(ras, params, m, v, accum, count, noise, lp_o, sh_degree, stats=True):
    from paper_2510_26358_amd.rasterizer import LifecycleParams
    lp = LifecycleParams(**lp_o.__dict__)
    st = (torch.from_numpy(accum).cuda(), torch.from_numpy(count).cuda()) if stats else None
    nz = torch.from_numpy(noise).cuda() if noise is not None else None
    p2, m2, v2, act = ras.lifecycle(_to_gpu(params, sh_degree), _to_gpu(m, sh_degree), _to_gpu(v, sh_degree), lp,
                                    stats=st, noise=nz)
    torch.cuda.synchronize()
    return _aos(p2), _aos(m2), _aos(v2), act.cpu().numpy().astype(np.int64)


def _compare_lifecycle(got, ref, params):
    gp, gm, gv, gact = got
    rp, rm, rv, ract = ref
    assert np.array_equal(gact, ract)
    n_out = len(rp["means"])
    print("n_in", len(ract), "n_out", n_out, "split", int((ract == olc.SPLIT).sum()),
          "clone", int((ract == olc.CLONE).sum()), "prune", int((ract == olc.PRUNE).sum()))
    assert len(gp["means"]) == n_out
    # moments and the untouched fields are exact copies (float32 in, float32 out)
    for k in NAMES:
        assert np.array_equal(gm[k], rm[k]), k
        assert np.array_equal(gv[k], rv[k]), k
    for k in ("quats", "sh"):
        assert np.array_equal(gp[k], rp[k]), k
    # logits: copies exact, reset values are float32 of logit(tau_reset)
    assert np.allclose(gp["opacity_logits"], rp["opacity_logits"], rtol=0, atol=1e-6)
    # children: float32 rotation of float32 inputs vs the float64 oracle (|eps| < 6, s < 1)
    dm = np.abs(gp["means"] - rp["means"])
    bound = 2e-6 * (1.0 + np.abs(rp["means"]) + 6.0 * np.exp(rp["log_scales"]).max(axis=1, keepdims=True))
    print("max |d mean| / bound", (dm / bound).max() if n_out else 0.0)
    assert np.all(dm <= bound)
    assert np.allclose(gp["log_scales"], rp["log_scales"], rtol=0, atol=4e-6)


@pytest.mark.parametrize("seed,n,deg,flags", [
    (311, 3000, 3, dict()),
    (312, 777, 1, dict(do_reset=True)),
    (313, 1500, 0, dict(do_prune=False)),
    (314, 2049, 2, dict(do_densify=False, do_reset=True)),
])
def test_lifecycle_step_matches_oracle(ras, seed, n, deg, flags):
    lp = olc.LifecycleParams(**flags)
    params, m, v, accum, count, noise = _lifecycle_inputs(seed, n, deg, lp)
    ref = olc.apply({k: a.astype(np.float64) for k, a in params.items()}, m, v, accum, count,
                    noise.astype(np.float64), lp)
    got = _run_lifecycle(ras, params, m, v, accum, count, noise if lp.do_densify else None, lp, deg,
                         stats=lp.do_densify)
    _compare_lifecycle(got, ref, params)


def test_lifecycle_step_at_full_size(ras):
    """The bench's Gaussian count (one million, SH degree 3)."""
    lp = olc.LifecycleParams(do_reset=True)
    n = 1 << 20
    params, m, v, accum, count, noise = _lifecycle_inputs(315, n, 3, lp)
    ref = olc.apply({k: a.astype(np.float64) for k, a in params.items()}, m, v, accum, count,
                    noise.astype(np.float64), lp)
    got = _run_lifecycle(ras, params, m, v, accum, count, noise, lp, 3)
    _compare_lifecycle(got, ref, params)


def test_lifecycle_edge_cases(ras):
    from paper_2510_26358_amd import _lib as L
    from paper_2510_26358_amd.rasterizer import LifecycleParams, SplatParams
    lp = olc.LifecycleParams()
    # empty input
    params, m, v, accum, count, noise = _lifecycle_inputs(316, 1, 1, lp)
    empty = {k: a[:0] for k, a in params.items()}
    got = _run_lifecycle(ras, empty, empty, empty, accum[:0], count[:0], noise[:0], lp, 1)
    assert len(got[0]["means"]) == 0 and len(got[3]) == 0
    # everything pruned
    params, m, v, accum, count, noise = _lifecycle_inputs(317, 300, 1, lp)
    params["opacity_logits"][:] = -10.0
    ref = olc.apply({k: a.astype(np.float64) for k, a in params.items()}, m, v, accum, count,
                    noise.astype(np.float64), lp)
    got = _run_lifecycle(ras, params, m, v, accum, count, noise, lp, 1)
    assert len(ref[0]["means"]) == 0
    _compare_lifecycle(got, ref, params)
    # densification needs the statistic and the noise; capacity below 2 N is refused
    g = _to_gpu(params, 1)
    with pytest.raises(RuntimeError):
        ras.lifecycle(g, g, g, LifecycleParams(), stats=None, noise=None)
    st = (torch.from_numpy(accum).cuda(), torch.from_numpy(count).cuda())
    with pytest.raises(RuntimeError):
        ras.lifecycle(g, g, g, LifecycleParams(), stats=st, noise=torch.from_numpy(noise).cuda(), capacity=599)
    assert L.AGS_ERR_INVALID_ARG < 0
