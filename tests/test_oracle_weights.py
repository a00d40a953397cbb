"""Pins for the oracle's discrepancy weights and distances (Alg. 1 line 4).

The default weight of frame f is the inverse of the frame's noise variance in
the Gaussian noise model of Sec. III-A1, sigma_f^2 = C_f exp(lambda t_f) / dt_f
(up to the global constant l^2, which cannot change a ranking), with the
unknown noise-free C replaced by the observed y floored at a fraction of the
voxel's maximum (the reading adopted where the paper is silent), t_f the frame
midpoint.  The L1 option of Sec. V weighs |y - x| by sqrt(w), the inverse
noise standard deviation.

Here the weights are built from that variance formula written out in the test
(frame bounds, midpoints and lengths from the frame schedule, numpy exp), and
the distances from oracle curves of the oracle's draws, summed in numpy.  A
wrong sign in the decay factor, the frame length on the wrong side, the frame
start in place of the midpoint, a wrong floor or w in place of sqrt(w) in the
L1 sum each fail one of these tests.
"""
import math

import numpy as np
import pytest

import workloads as W

H = 0.2


def _sched_bounds(sched):
    """fp32 frame bounds, and in FP64 the bounds as grid nodes t_k = k h
    (h the fp32 step), the frame midpoints and the frame lengths."""
    ft = W.frame_times(sched)
    h = float(np.float32(H))
    tau = np.rint(ft.astype(np.float64) / h) * h
    return ft, tau, 0.5 * (tau[1:] + tau[:-1]), np.diff(tau)


def _variance(c, tmid, dt, lam):
    """Noise variance of Sec. III-A1 without its global constant."""
    return c * np.exp(lam * tmid) / dt


@pytest.mark.parametrize("lam", [math.log(2.0) / 109.8, math.log(2.0) / 20.4, 0.1])
@pytest.mark.parametrize("sched", [W.SCHED_22x60, W.SCHED_30x50, W.SCHED_40x90])
def test_weights_are_inverse_noise_variance(ora, sched, lam):
    ft, _, tmid, dt = _sched_bounds(sched)
    F = ft.size - 1
    _, cp = W.grid(H, float(ft[-1]))
    rng = np.random.default_rng(F)
    # positive curves whose every frame lies above the floor
    y = rng.uniform(0.5, 20.0, size=(8, F)).astype(np.float32)
    for v in range(y.shape[0]):
        w = ora.weights(y[v], ft, H, cp.size, lam=lam)
        prod = w * _variance(y[v].astype(np.float64), tmid, dt, lam)
        assert np.all(np.isfinite(prod)) and prod.min() > 0
        # one constant for every frame: w is the inverse variance up to scale
        assert np.ptp(prod) <= 1e-13 * prod.mean(), (v, prod)
        # the constant is 1: the oracle drops exactly the global l^2
        assert prod.mean() == pytest.approx(1.0, rel=1e-13)


@pytest.mark.parametrize("floor", [0.01, 0.05, 0.3])
def test_weight_floor_replaces_small_and_negative_frames(ora, floor):
    sched = W.SCHED_22x60
    ft, _, tmid, dt = _sched_bounds(sched)
    F = ft.size - 1
    _, cp = W.grid(H, float(ft[-1]))
    lam = math.log(2.0) / 109.8
    y = np.linspace(2.0, 40.0, F).astype(np.float32)
    small = [0, 3, 7, 12]
    y[small] = np.float32([1e-4, -3.0, 0.0, 0.5 * floor * float(y.max())])
    w = ora.weights(y, ft, H, cp.size, lam=lam, floor=floor)
    den = np.maximum(y.astype(np.float64), floor * float(y.max()))
    prod = w * _variance(den, tmid, dt, lam)
    assert np.ptp(prod) <= 1e-13 * prod.mean()
    assert prod.mean() == pytest.approx(1.0, rel=1e-13)
    # floored frames: weight = dt exp(-lam t) / (floor * max y) exactly
    fl = floor * float(y.max())
    for f in small:
        assert w[f] == pytest.approx(dt[f] * math.exp(-lam * tmid[f]) / fl, rel=1e-13)
    # frames above the floor do not see it
    big = np.nonzero(y.astype(np.float64) > fl)[0]
    assert big.size >= F // 2
    assert np.allclose(w[big] * _variance(y[big].astype(np.float64), tmid[big], dt[big], lam), 1.0, rtol=1e-13)


def _draw_curves(ora, models, boxes, seed, v, n_draws, cp, ft):
    """Oracle draws (pinned bit for bit against rocRAND's Philox) and their
    oracle curves (pinned against closed forms) for every g = m n_draws + i."""
    M = len(models)
    g = np.arange(M * n_draws)
    m, i = g // n_draws, g % n_draws
    _, _, th = ora.draws(models, boxes, seed, np.full(g.size, v), i, m)
    x = np.empty((g.size, ft.size - 1))
    for mm, model in enumerate(models):
        sel = m == mm
        x[sel] = ora.simulate(model, th[sel], cp, H, ft)
    return x


@pytest.mark.parametrize("l1", [False, True])
def test_distances_are_the_weighted_sums(ora, l1):
    """voxel_distances and the accepted distances of infer equal
    sum_f w_f r_f^2 (L2) or sum_f sqrt(w_f) |r_f| (L1), r = y - x, with w the
    inverse noise variance built in this test."""
    sched = W.SCHED_22x60
    ft, _, tmid, dt = _sched_bounds(sched)
    _, cp = W.grid(H, float(ft[-1]))
    lam = math.log(2.0) / 109.8
    models = [W.M_2TCM_IRR, W.M_1TCM]
    boxes = W.box_array(models)
    th, _ = W.CFG_SMALL.truth(3)
    clean = ora.simulate(W.M_2TCM_IRR, th, cp, H, ft)
    y = W.add_noise(clean, ft, np.random.default_rng(4).standard_normal(clean.shape))
    y[1, :3] = np.float32(1e-3)  # a few floored frames
    n_draws, p, seed = 400, 0.02, 19
    res = ora.infer(y, ft, cp, H, models, boxes, n_draws, p, seed, l1=l1)
    for v in range(y.shape[0]):
        yv = y[v].astype(np.float64)
        w = 1.0 / _variance(np.maximum(yv, 0.01 * yv.max()), tmid, dt, lam)
        x = _draw_curves(ora, models, boxes, seed, v, n_draws, cp, ft)
        r = yv - x
        d = (np.sqrt(w) * np.abs(r)).sum(axis=1) if l1 else (w * r * r).sum(axis=1)
        d_ora = ora.voxel_distances(y[v], ft, cp, H, models, boxes, n_draws, seed, v, l1=l1)
        assert np.allclose(d_ora, d, rtol=1e-11, atol=0), np.abs(d_ora / d - 1).max()
        order = np.lexsort((np.arange(d.size), d))[:res["n"]]
        assert np.array_equal(res["accept_idx"][v], order)
        assert np.allclose(res["accept_dist"][v], d[order], rtol=1e-11, atol=0)


def test_caller_weights_enter_as_given(ora):
    """With caller weights the distance is sum w r^2 / sum sqrt(w) |r| of
    exactly those weights (fp32 promoted)."""
    sched = W.SCHED_22x60
    ft, _, _, _ = _sched_bounds(sched)
    _, cp = W.grid(H, float(ft[-1]))
    models = [W.M_2TCM_IRR]
    boxes = W.box_array(models)
    th, _ = W.CFG_SMALL.truth(1)
    y = ora.simulate(W.M_2TCM_IRR, th, cp, H, ft).astype(np.float32)
    wv = np.random.default_rng(8).uniform(0.0, 3.0, size=ft.size - 1).astype(np.float32)
    x = _draw_curves(ora, models, boxes, 5, 0, 300, cp, ft)
    r = y[0].astype(np.float64) - x
    w = wv.astype(np.float64)
    for l1, d in ((False, (w * r * r).sum(1)), (True, (np.sqrt(w) * np.abs(r)).sum(1))):
        d_ora = ora.voxel_distances(y[0], ft, cp, H, models, boxes, 300, 5, 0, l1=l1, weights_v=wv)
        assert np.allclose(d_ora, d, rtol=1e-11, atol=0)
