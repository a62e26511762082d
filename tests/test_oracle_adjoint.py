"""The oracle's two gradient statements agree: torch float64 autograd through projection and
compositing (oracle.render) and the hand-derived chain rule (oracle.adjoint), for the
upstream-gradient objective sum_p g_C.C + g_D D + g_A A with the same frozen decisions, to
1e-9 relative, on scenes that exercise the alpha clamp, the colour clamp at 0, the
field-of-view clamp of the Jacobian, a non-identity view pose and a second view."""
import math

import numpy as np

from oracle.adjoint import upstream_grads
from oracle.render import loss_and_grads
from oracle.settings import RenderSettings
from tests.oracle_helpers import random_scene

NAMES = ["means", "log_scales", "quats", "opacity_logits", "sh"]


def _upstream(rng, sc):
    return [{"rgb": rng.normal(size=(3, c.height, c.width)), "depth": rng.normal(size=(c.height, c.width)),
             "alpha": rng.normal(size=(c.height, c.width))} for c in sc.cameras]


def _check(sc, seed):
    rng = np.random.default_rng(seed)
    up = _upstream(rng, sc)
    s = RenderSettings()
    ref = loss_and_grads(sc, s, upstream=up)
    got = upstream_grads(sc, up, s, decisions=ref["decisions"])
    for k in NAMES:
        r, g = np.asarray(ref["grads"][k]), got["grads"][k]
        scale = max(np.abs(r).max(), 1e-300)
        err = np.abs(g - r).max() / scale
        print(k, "max |diff| / max |ref|", err)
        assert err <= 1e-9, k
    err = np.abs(got["pose"] - ref["pose"]).max() / np.abs(ref["pose"]).max()
    print("pose", err)
    assert err <= 1e-9


def test_adjoint_matches_autograd_two_views_sh3():
    _check(random_scene(501, n=80, sh_degree=3, n_views=2, width=40, height=30, f=45.0), 5011)


def test_adjoint_matches_autograd_with_the_clamps_active():
    sc = random_scene(502, n=60, sh_degree=2, n_views=1, width=36, height=28, f=40.0)
    # alpha clamp: nearly opaque splats, wide enough for pixel centres to fall where
    # o e^power > 0.99
    sc.opacity_logits[:10] = 7.0
    sc.log_scales[:10] = math.log(0.6)
    # colour clamp at 0: strongly negative DC for some channels
    sc.sh[10:20, 0, 1] = -4.0
    # field-of-view clamp: large splats centred outside 1.3 half-widths that still cover pixels
    lim = 1.3 * 36 / (2 * 40.0)
    for k, sx in enumerate((1.6, -1.7, 1.5)):
        sc.means[20 + k] = [sx * lim * 3.0, 0.1 * k, 3.0]
        sc.log_scales[20 + k] = [math.log(1.2), math.log(0.4), math.log(0.5)]
        sc.opacity_logits[20 + k] = 2.0
    # the three branches are taken
    from oracle.render import render
    out = render(sc)[0]
    dec, pr = out["dec"], out["proj"]
    contrib = np.unique(dec.idx[dec.idx >= 0])
    assert dec.clamped.sum() > 0
    assert (pr["rgb"].detach().numpy()[contrib] == 0).any(1).sum() > 0
    xc = sc.means[contrib] @ sc.cameras[0].R.T + sc.cameras[0].t
    assert (np.abs(xc[:, 0] / xc[:, 2]) > lim).sum() > 0
    _check(sc, 5021)
