"""Pins for the lifecycle oracle (Sec. III-B: pruning, gradient-driven split / duplicate,
opacity reset) and for the densification statistic the backward accumulates: hand-built
cases for every rule and the precedence between them, invariants of the outputs (order,
counts, copies exact, split children distributed as the parent Gaussian), and the
statistic against finite differences of the loss in the projected centre."""
import math

import numpy as np

from oracle.lifecycle import CLONE, KEEP, PRUNE, SPLIT, LifecycleParams, apply, classify, quat_rotation
from oracle.render import loss_and_grads
from oracle.settings import RenderSettings
from tests.oracle_helpers import random_scene


def _logit(o):
    return math.log(o / (1 - o))


def _case():
    # one Gaussian per rule; sizes are exp(max log-scale)
    ls = np.log(np.array([
        [0.02, 0.01, 0.01],    # 0 keep (cool)
        [0.02, 0.01, 0.01],    # 1 prune: faint
        [0.5, 0.01, 0.01],     # 2 prune: too large
        [1e-5, 1e-5, 2e-5],    # 3 prune: too small
        [0.05, 0.01, 0.01],    # 4 split: hot and s > kappa
        [0.008, 0.002, 0.002],  # 5 clone: hot and s <= 2 s_init
        [0.009, 0.002, 0.002],  # 6 keep: hot but 2 s_init < s <= kappa
        [0.05, 0.01, 0.01],    # 7 keep: hot but never seen (count 0)
        [0.02, 0.01, 0.01],    # 8 reset candidate (0.01 <= o < 0.05)
    ]))
    o = np.array([0.5, 0.005, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.03])
    logits = np.array([_logit(x) for x in o])
    accum = np.array([0.0, 1.0, 1.0, 1.0, 0.5, 0.3, 0.3, 0.0, 0.0])
    count = np.array([2, 2, 2, 2, 2, 2, 2, 0, 1])
    return ls, logits, accum, count


def test_classification_rules_and_precedence():
    ls, logits, accum, count = _case()
    lp = LifecycleParams(grad_threshold=0.1, kappa=0.01, s_init=0.0044, do_reset=True, tau_reset=0.05)
    act, reset = classify(ls, logits, accum, count, lp)
    assert list(act) == [KEEP, PRUNE, PRUNE, PRUNE, SPLIT, CLONE, KEEP, KEEP, KEEP]
    assert list(np.nonzero(reset)[0]) == [8]
    # switches
    act2, _ = classify(ls, logits, accum, count, LifecycleParams(do_prune=False, grad_threshold=0.1, kappa=0.01,
                                                                    s_init=0.0044))
    assert act2[1] == SPLIT and act2[2] == SPLIT and act2[4] == SPLIT  # nothing pruned: hot and large
    act3, _ = classify(ls, logits, accum, count, LifecycleParams(do_densify=False))
    assert not np.isin(act3, [SPLIT, CLONE]).any()


def test_apply_outputs_order_copies_and_children():
    ls, logits, accum, count = _case()
    n = len(logits)
    rng = np.random.default_rng(3)
    params = {"means": rng.normal(size=(n, 3)), "log_scales": ls, "quats": rng.normal(size=(n, 4)),
              "opacity_logits": logits, "sh": rng.normal(size=(n, 16, 3))}
    m = {k: rng.normal(size=np.shape(a)) for k, a in params.items()}
    v = {k: rng.random(size=np.shape(a)) for k, a in params.items()}
    noise = rng.normal(size=(n, 2, 3))
    lp = LifecycleParams(grad_threshold=0.1, kappa=0.01, s_init=0.0044, do_reset=True, tau_reset=0.05)
    out, om, ov, act = apply(params, m, v, accum, count, noise, lp)
    # output rows: 0, 4a, 4b, 5, 5', 6, 7, 8
    assert len(out["means"]) == 8
    src = [0, 4, 4, 5, 5, 6, 7, 8]
    for k in ("quats", "sh"):
        assert np.array_equal(out[k], np.asarray(params[k])[src])
    assert np.array_equal(out["means"][[0, 3, 4, 5, 6, 7]], params["means"][[0, 5, 5, 6, 7, 8]])
    # duplicate: exact copy, new optimiser state zero; survivors keep theirs
    assert np.array_equal(om["means"][3], m["means"][5]) and not om["means"][4].any()
    assert not om["sh"][[1, 2]].any() and not ov["quats"][[1, 2]].any()
    # children of 4: mean + R diag(s) eps, scales / 1.6
    R = quat_rotation(params["quats"][[4]])[0]
    s = np.exp(ls[4])
    for c in range(2):
        assert np.allclose(out["means"][1 + c], params["means"][4] + R @ (s * noise[4, c]), rtol=0, atol=1e-14)
        assert np.allclose(out["log_scales"][1 + c], ls[4] - math.log(1.6), rtol=0, atol=1e-14)
    # reset
    assert math.isclose(out["opacity_logits"][7], _logit(0.05), rel_tol=1e-12)
    assert out["opacity_logits"][0] == logits[0]


def test_split_children_are_samples_of_the_parent():
    """Children of one parent over many noise draws: mean mu, covariance R S S R^T (the
    parent's 3D covariance) -- the Monte Carlo pins R and the scale order."""
    rng = np.random.default_rng(5)
    n = 20000
    q = np.tile(rng.normal(size=(1, 4)), (n, 1))
    ls = np.tile(np.log([[0.05, 0.02, 0.01]]), (n, 1))
    params = {"means": np.tile([[1.0, 2.0, 3.0]], (n, 1)), "log_scales": ls, "quats": q,
              "opacity_logits": np.zeros(n), "sh": np.zeros((n, 1, 3))}
    z = {k: np.zeros_like(a) for k, a in params.items()}
    out, _, _, act = apply(params, z, z, np.ones(n), np.ones(n, np.int64), rng.normal(size=(n, 2, 3)),
                           LifecycleParams(grad_threshold=0.1, kappa=0.01))
    assert (act == SPLIT).all()
    x = out["means"]
    R = quat_rotation(q[:1])[0]
    cov = R @ np.diag(np.exp(ls[0]) ** 2) @ R.T
    assert np.allclose(x.mean(0), [1, 2, 3], atol=5 * 0.05 / math.sqrt(2 * n))
    assert np.allclose(np.cov(x.T), cov, rtol=0, atol=0.05 * np.abs(cov).max())


def test_densification_statistic_is_the_centre_gradient():
    """Stats = sum over views of |dL/d(u, v)|: checked against central differences of the
    loss in a rigid pixel shift of one Gaussian's projection (moving its mean along the
    camera's x and y axes by h z / f moves u, v by h)."""
    sc = random_scene(81, n=30, n_views=1, width=32, height=24, f=40.0)
    s = RenderSettings()
    r = loss_and_grads(sc, s, lam=0.5, stats=True)
    st = r["stats"]
    assert st["count"].max() <= 1 and st["count"].sum() > 0
    cam = sc.cameras[0]
    R = cam.R.astype(np.float64)
    i = int(np.argmax(st["grad_accum"]))
    z = (R @ sc.means[i] + cam.t)[2]
    from oracle.render import frozen_objective
    g = []
    for axis, f in ((0, cam.fx), (1, cam.fy)):
        h = 1e-4
        d = R[axis] * h * z / f  # world displacement moving u (or v) by h to first order
        old = sc.means[i].copy()
        sc.means[i] = old + d
        lp = frozen_objective(sc, r["decisions"], s, lam=0.5)
        sc.means[i] = old - d
        lm = frozen_objective(sc, r["decisions"], s, lam=0.5)
        sc.means[i] = old
        g.append((lp - lm) / (2 * h))
    # a mean shift along the camera axes also moves the depth / J slightly; the centre
    # gradient dominates, so compare to 2 %
    assert math.isclose(st["grad_accum"][i], math.hypot(*g), rel_tol=2e-2), (st["grad_accum"][i], g)
