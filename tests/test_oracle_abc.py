"""Pins for the oracle's rejection ABC (Alg. 1 and the fixed-budget variant of
Sec. II-C) and its posterior summaries (Eq. (6), Sec. II-D3, Sec. III-B2).

Checked against:
  * brute-force ranking of every draw's distance (tiny inputs);
  * fully degenerate priors (every distance ties -> lowest indices win);
  * p = 1 (every draw accepted -> plain sample moments of the draws);
  * a 1-parameter problem whose simulated TAC is linear in the parameter, where
    the accepted set is exactly the draws inside an interval known in closed
    form, and whose ABC target is the uniform distribution on that interval;
  * a nonlinear 1-parameter problem against a dense grid of the prior;
  * two identical models (P = 1/2);
  * invariance of the accepted set to a global weight scale;
  * invalid voxels -> NaN outputs; the global voxel offset.
"""
import numpy as np
import pytest

import workloads as W

H = 0.2


def _setup(sched=W.SCHED_22x60):
    ft = W.frame_times(sched)
    t_end = float(np.sum(sched))
    _, cp = W.grid(H, t_end)
    return ft, cp


def _box(models, fixed=None, free=None):
    b = W.box_array(models)
    if fixed:
        for (m, s), val in fixed.items():
            b[m, s] = (val, val)
    if free:
        for (m, s), rng in free.items():
            b[m, s] = rng
    return b


def _observed(ora, model, theta, ft, cp, seed=7, level=0.05):
    clean = ora.simulate(model, theta, cp, H, ft)
    eps = np.random.default_rng(seed).standard_normal(clean.shape)
    return W.add_noise(clean, ft, eps, level=level)


def test_accept_count():
    import oracle
    assert oracle.accept_count(2000, 0.01) == 20
    assert oracle.accept_count(100000, 0.001) == 100
    assert oracle.accept_count(3, 0.999) == 2
    assert oracle.accept_count(10, 0.3) == 3      # 10 * 0.3 = 2.9999999999999996 in FP64
    assert oracle.accept_count(10, 0.05) == 0     # n < 1
    assert oracle.accept_count(10, 0.0) == 0
    assert oracle.accept_count(10, 1.0) == 10
    assert oracle.accept_count(10, 1.5) == 0


@pytest.mark.parametrize("l1", [False, True])
def test_selection_matches_brute_force(ora, l1):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_1TCM], dtype=np.uint32)
    boxes = W.box_array(list(models))
    th, _ = W.CFG_SMALL.truth(3)
    y = _observed(ora, W.M_2TCM_IRR, th, ft, cp)
    n_draws, p = 150, 0.05
    res = ora.infer(y, ft, cp, H, models, boxes, n_draws, p, 31, l1=l1)
    n = res["n"]
    assert n == 15
    for v in range(3):
        d = ora.voxel_distances(y[v], ft, cp, H, models, boxes, n_draws, 31, v, l1=l1)
        keys = list(zip(d, range(d.size)))
        rank = np.array([sum(1 for k2 in keys if k2 < k) for k in keys])   # O(N^2) ranking
        order = np.argsort(rank)
        assert np.array_equal(res["accept_idx"][v], order[:n])
        assert np.array_equal(res["accept_dist"][v], d[order[:n]])
        assert res["threshold"][v] == d[order[n - 1]] and res["next_dist"][v] == d[order[n]]


def test_degenerate_prior_ties_go_to_lowest_index(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_2TCM_IRR], dtype=np.uint32)
    th = np.array([0.4, 0.2, 0.05, 0.0, 0.04])
    boxes = np.zeros((2, 8, 2))
    for m in range(2):
        for s in range(5):
            boxes[m, s] = (th[s], th[s])
    y = _observed(ora, W.M_2TCM_IRR, W.CFG_SMALL.truth(2)[0], ft, cp)
    res = ora.infer(y, ft, cp, H, models, boxes, 100, 0.3, 5)
    n = res["n"]
    assert n == 60
    for v in range(2):
        assert np.array_equal(res["accept_idx"][v], np.arange(n))
        assert np.all(res["accept_dist"][v] == res["accept_dist"][v][0])
    assert np.all(res["model_prob"][:, 0] == 1.0) and np.all(res["model_prob"][:, 1] == 0.0)
    mom = res["moments"]
    for s in (0, 1, 2, 4):
        assert np.all(mom[:, 0, s, 0] == np.float64(np.float32(th[s]))) and np.all(mom[:, 0, s, 1] == 0.0)
    assert np.all(np.isnan(mom[:, 1]))                # a model with no accepted draw


def test_p1_gives_sample_moments_of_all_draws(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_2TCM_REV], dtype=np.uint32)
    boxes = W.box_array(list(models))
    y = _observed(ora, W.M_2TCM_IRR, W.CFG_SMALL.truth(2)[0], ft, cp)
    n_draws = 400
    res = ora.infer(y, ft, cp, H, models, boxes, n_draws, 1.0, 77, voxel_offset=10)
    assert res["n"] == 800
    for v in range(2):
        for m in range(2):
            _, _, theta = ora.draws(models, boxes, 77, np.full(n_draws, v + 10), np.arange(n_draws),
                                    np.full(n_draws, m))
            t = theta.astype(np.float64)
            t[:, 5] = t[:, 0] * t[:, 2] / (t[:, 1] + t[:, 2])
            for s in (0, 1, 2, 3, 4, 5):
                if m == 0 and s == 3:
                    assert np.isnan(res["moments"][v, m, s]).all()
                    continue
                assert res["moments"][v, m, s, 0] == pytest.approx(t[:, s].mean(), rel=1e-12)
                assert res["moments"][v, m, s, 1] == pytest.approx(t[:, s].var(ddof=1), rel=1e-10)
                if s != 5:   # prior moments of a uniform box
                    lo, hi = boxes[m, s]
                    se = (hi - lo) / np.sqrt(12 * n_draws)
                    assert abs(res["moments"][v, m, s, 0] - 0.5 * (lo + hi)) < 4.5 * se
            assert res["model_prob"][v, m] == 0.5


def test_linear_one_parameter_target_is_exact_interval(ora):
    # K1 free, everything else fixed: the simulated TAC is c0 + K1 g exactly.
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR], dtype=np.uint32)
    fixed = {1: 0.25, 2: 0.06, 4: 0.05}
    boxes = _box([W.M_2TCM_IRR], fixed={(0, s): v for s, v in fixed.items()})
    base = np.full((3, 8), np.nan)
    for r, k1 in enumerate((0.0, 1.0, 0.37)):
        base[r, [0, 1, 2, 4]] = (k1, fixed[1], fixed[2], fixed[4])
    x = ora.simulate(W.M_2TCM_IRR, base, cp, H, ft)
    c0, g = x[0], x[1] - x[0]
    assert np.allclose(x[2], c0 + 0.37 * g, rtol=1e-12)        # linearity in K1
    truth = base[2:3].astype(np.float32)
    y = _observed(ora, W.M_2TCM_IRR, truth, ft, cp, seed=3)
    w = np.linspace(0.5, 2.0, ft.size - 1).astype(np.float32)[None, :]
    n_draws, p = 100_000, 0.01
    res = ora.infer(y, ft, cp, H, models, boxes, n_draws, p, 2024, weights=w)
    n, hthr = res["n"], res["threshold"][0]
    wd, yd = w[0].astype(np.float64), y[0].astype(np.float64)
    A, B = np.sum(wd * g * g), np.sum(wd * g * (yd - c0))
    C = np.sum(wd * (yd - c0) ** 2)
    khat, dmin = B / A, C - B * B / A
    r = np.sqrt((hthr - dmin) / A)
    lo, hi = khat - r, khat + r
    assert 0.01 < lo and hi < 1.0                              # interval inside the box
    _, _, th_all = ora.draws(models, boxes, 2024, np.zeros(n_draws), np.arange(n_draws), np.zeros(n_draws))
    k1 = th_all[:, 0].astype(np.float64)
    acc = k1[res["accept_idx"][0]]
    tol = 1e-9 * (hi - lo)
    assert acc.min() >= lo - tol and acc.max() <= hi + tol     # accepted draws lie in the interval
    inside = np.sum((k1 > lo + tol) & (k1 < hi - tol))
    assert n - 2 <= inside <= n                                # and every draw inside it is accepted
    mom = res["moments"][0, 0, 0]
    L = hi - lo
    assert abs(mom[0] - 0.5 * (lo + hi)) < 4 * L / np.sqrt(12 * n)
    assert mom[1] == pytest.approx(L * L / 12, rel=0.15)


@pytest.mark.slow
def test_nonlinear_one_parameter_matches_grid_target(ora):
    # k2 free: the ABC target is the prior restricted to {d <= h_p} (noise-free
    # simulations), computed on a dense grid of the prior.
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR], dtype=np.uint32)
    fixed = {0: 0.5, 2: 0.05, 4: 0.05}
    boxes = _box([W.M_2TCM_IRR], fixed={(0, s): v for s, v in fixed.items()})
    truth = np.full((1, 8), np.nan, dtype=np.float32)
    truth[0, [0, 1, 2, 4]] = (0.5, 0.3, 0.05, 0.05)
    y = _observed(ora, W.M_2TCM_IRR, truth, ft, cp, seed=11)
    G = 200_000
    lo, hi = boxes[0, 1]
    k2 = lo + (np.arange(G) + 0.5) / G * (hi - lo)
    grid = np.full((G, 8), np.nan)
    grid[:, 0], grid[:, 1], grid[:, 2], grid[:, 4] = fixed[0], k2, fixed[2], fixed[4]
    xg = ora.simulate(W.M_2TCM_IRR, grid, cp, H, ft)
    w = ora.weights(y[0], ft, H, cp.size)
    d = np.sum(w * (y[0].astype(np.float64) - xg) ** 2, axis=1)
    p = 0.01
    hp = np.quantile(d, p)
    sel = k2[d <= hp]
    t_mean, t_sd = sel.mean(), sel.std()
    res = ora.infer(y, ft, cp, H, models, boxes, 100_000, p, 99)
    n = res["n"]
    se = t_sd / np.sqrt(n)
    assert abs(res["moments"][0, 0, 1, 0] - t_mean) < 4 * se
    assert res["moments"][0, 0, 1, 1] == pytest.approx(t_sd ** 2, rel=0.2)


def test_identical_models_have_probability_half(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_2TCM_REV], dtype=np.uint32)
    boxes = _box(list(models), fixed={(1, 3): 0.0})     # k4 = 0: REV is IRR
    th, _ = W.CFG_SMALL.truth(8)
    y = _observed(ora, W.M_2TCM_IRR, th, ft, cp)
    res = ora.infer(y, ft, cp, H, models, boxes, 20_000, 0.0125, 8, nthreads=4)
    n = res["n"]
    assert n == 500
    pr = res["model_prob"][:, 0]
    se = np.sqrt(0.25 / n)
    assert np.all(np.abs(pr - 0.5) < 4 * se)
    assert abs(pr.mean() - 0.5) < 4 * se / np.sqrt(8)
    assert np.allclose(res["model_prob"].sum(axis=1), 1.0)


def test_strongly_reversible_data_prefers_reversible_model(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_2TCM_REV], dtype=np.uint32)
    boxes = W.box_array(list(models))
    th = np.full((4, 8), np.nan, dtype=np.float32)
    th[:, [0, 1, 2, 3, 4]] = (0.6, 0.3, 0.25, 0.1, 0.05)
    clean = ora.simulate(W.M_2TCM_REV, th, cp, H, ft)
    y = W.add_noise(clean, ft, np.random.default_rng(1).standard_normal(clean.shape), level=0.005)
    res = ora.infer(y, ft, cp, H, models, boxes, 20_000, 0.005, 4)
    assert np.all(res["model_prob"][:, 1] > 0.5)


def test_weight_scale_does_not_change_accepted_set(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR], dtype=np.uint32)
    boxes = W.box_array(list(models))
    y = _observed(ora, W.M_2TCM_IRR, W.CFG_SMALL.truth(4)[0], ft, cp)
    w = np.stack([ora.weights(yv, ft, H, cp.size) for yv in y]).astype(np.float32)
    a = ora.infer(y, ft, cp, H, models, boxes, 3000, 0.01, 5, weights=w)
    b = ora.infer(y, ft, cp, H, models, boxes, 3000, 0.01, 5, weights=(w * np.float32(3.7)))
    assert np.array_equal(a["accept_idx"], b["accept_idx"])
    assert np.allclose(a["moments"], b["moments"], rtol=1e-14, equal_nan=True)


def test_invalid_voxels_give_nan_and_offset_is_global(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR], dtype=np.uint32)
    boxes = W.box_array(list(models))
    y = _observed(ora, W.M_2TCM_IRR, W.CFG_SMALL.truth(6)[0], ft, cp)
    y[1, 3] = np.nan
    y[2] = -1.0
    res = ora.infer(y, ft, cp, H, models, boxes, 500, 0.02, 9)
    for v in (1, 2):
        assert np.isnan(res["moments"][v]).all() and np.isnan(res["model_prob"][v]).all()
    assert np.isfinite(res["model_prob"][[0, 3, 4, 5]]).all()
    sub = ora.infer(y[3:], ft, cp, H, models, boxes, 500, 0.02, 9, voxel_offset=3)
    assert np.array_equal(sub["accept_idx"], res["accept_idx"][3:])
    assert np.array_equal(sub["moments"], res["moments"][3:], equal_nan=True)
    # the thread count does not change the result
    par = ora.infer(y, ft, cp, H, models, boxes, 500, 0.02, 9, nthreads=3)
    assert np.array_equal(par["accept_idx"], res["accept_idx"])


# ---------------------------------------------------------------------------
# Shared-bank form (Alg. 1 as printed: one bank of draws for all voxels)
# ---------------------------------------------------------------------------
def test_bank_draws_and_curves(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_2TCM_REV], dtype=np.uint32)
    boxes = W.box_array(list(models))
    th, x = ora.bank(models, boxes, 300, 42, cp, H, ft)
    # bank draw i of model m is the Philox draw of counter (i, 0, 1, m<<16|blk)
    m = np.repeat([0, 1], 300)
    i = np.tile(np.arange(300), 2)
    _, _, th2 = ora.draws(models, boxes, 42, np.zeros(600), i, m, stream=1)
    assert np.array_equal(th.view(np.uint32), th2.view(np.uint32))
    assert np.array_equal(x[:300], ora.simulate(W.M_2TCM_IRR, th[:300], cp, H, ft))
    assert np.array_equal(x[300:], ora.simulate(W.M_2TCM_REV, th[300:], cp, H, ft))


def test_bank_selection_matches_brute_force(ora):
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR, W.M_1TCM], dtype=np.uint32)
    boxes = W.box_array(list(models))
    y = _observed(ora, W.M_2TCM_IRR, W.CFG_SMALL.truth(4)[0], ft, cp)
    y[2] = y[1]                                    # identical voxels share the bank's answer
    n_draws, p = 200, 0.05
    res = ora.infer_bank(y, ft, cp, H, models, boxes, n_draws, p, 17)
    _, x = ora.bank(models, boxes, n_draws, 17, cp, H, ft)
    for v in range(4):
        w = ora.weights(y[v], ft, H, cp.size)
        d = np.sum(w * (y[v].astype(np.float64) - x) ** 2, axis=1)
        keys = list(zip(d, range(d.size)))
        rank = np.array([sum(1 for k2 in keys if k2 < k) for k in keys])
        order = np.argsort(rank)
        assert np.array_equal(res["accept_idx"][v], order[:res["n"]])
        assert np.allclose(res["accept_dist"][v], d[order[:res["n"]]], rtol=1e-13)
    assert np.array_equal(res["accept_idx"][1], res["accept_idx"][2])
    assert np.array_equal(res["moments"][1], res["moments"][2], equal_nan=True)


def test_bank_linear_target_interval(ora):
    # the exact-interval pin of the per-voxel form, for the shared bank
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR], dtype=np.uint32)
    fixed = {1: 0.25, 2: 0.06, 4: 0.05}
    boxes = _box([W.M_2TCM_IRR], fixed={(0, s): v for s, v in fixed.items()})
    base = np.full((2, 8), np.nan)
    for r, k1 in enumerate((0.0, 1.0)):
        base[r, [0, 1, 2, 4]] = (k1, fixed[1], fixed[2], fixed[4])
    xb = ora.simulate(W.M_2TCM_IRR, base, cp, H, ft)
    c0, g = xb[0], xb[1] - xb[0]
    truth = np.full((3, 8), np.nan, dtype=np.float32)
    truth[:, [0, 1, 2, 4]] = [(0.3, 0.25, 0.06, 0.05), (0.5, 0.25, 0.06, 0.05), (0.8, 0.25, 0.06, 0.05)]
    y = _observed(ora, W.M_2TCM_IRR, truth, ft, cp, seed=5)
    n_draws, p = 50_000, 0.01
    res = ora.infer_bank(y, ft, cp, H, models, boxes, n_draws, p, 9)
    th, _ = ora.bank(models, boxes, n_draws, 9, cp, H, ft)
    k1 = th[:, 0].astype(np.float64)
    for v in range(3):
        w = ora.weights(y[v], ft, H, cp.size)
        yd = y[v].astype(np.float64)
        A, B = np.sum(w * g * g), np.sum(w * g * (yd - c0))
        C = np.sum(w * (yd - c0) ** 2)
        r = np.sqrt((res["threshold"][v] - (C - B * B / A)) / A)
        lo, hi = B / A - r, B / A + r
        acc = k1[res["accept_idx"][v]]
        tol = 1e-6 * (hi - lo)   # the edges carry the cancellation of C - B^2/A
        assert acc.min() >= lo - tol and acc.max() <= hi + tol
        assert res["n"] - 2 <= np.sum((k1 > lo + tol) & (k1 < hi - tol)) <= res["n"]


def test_bad_caller_weights_invalidate_the_voxel(ora):
    """Reading R10: a negative or non-finite caller weight makes the voxel
    invalid (NaN outputs, nothing accepted); a zero weight is allowed."""
    ft, cp = _setup()
    models = np.array([W.M_2TCM_IRR], dtype=np.uint32)
    boxes = W.box_array(list(models))
    y = _observed(ora, W.M_2TCM_IRR, W.CFG_SMALL.truth(7)[0][:5], ft, cp)
    w = np.stack([ora.weights(yv, ft, H, cp.size) for yv in y]).astype(np.float32)
    w[1, 3] = -0.5
    w[2, 0] = np.inf
    w[3, 5] = 0.0
    res = ora.infer(y, ft, cp, H, models, boxes, 500, 0.02, 9, weights=w)
    for v in (1, 2):
        assert np.isnan(res["moments"][v]).all() and np.isnan(res["model_prob"][v]).all()
        assert (res["accept_idx"][v] == -1).all()
    for v in (0, 3, 4):
        assert np.isfinite(res["moments"][v, 0, [0, 1, 2, 4, 5], 0]).all()
    rb = ora.infer_bank(y, ft, cp, H, list(models), boxes, 500, 0.02, 9, weights=w)
    for v in (1, 2):
        assert np.isnan(rb["moments"][v]).all() and (rb["accept_idx"][v] == -1).all()
    assert np.isfinite(rb["moments"][3, 0, 5, 0])


def test_summarize_set_reproduces_the_oracle_summaries(ora):
    """The reduction applied to an explicit set (used for voxels whose GPU set
    differs at the threshold) equals the oracle's own summaries of its own
    sets, per-voxel draws and shared bank; and it follows the set it is given."""
    ft, cp = _setup()
    models = [W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV]
    boxes = W.box_array(models)
    th, _ = W.CFG_SMALL.truth(4)
    y = _observed(ora, W.M_2TCM_IRR, th, ft, cp)
    res = ora.infer(y, ft, cp, H, models, boxes, 300, 0.05, 23, voxel_offset=11)
    for v in range(y.shape[0]):
        mom, pr = ora.summarize_set(res["accept_idx"][v][::-1], models, boxes, 300, 23, v_global=11 + v)
        assert np.allclose(mom, res["moments"][v], rtol=1e-12, atol=1e-15, equal_nan=True)
        assert np.array_equal(pr, res["model_prob"][v])
    rb = ora.infer_bank(y, ft, cp, H, models, boxes, 300, 0.05, 23)
    th_b, _ = ora.bank(models, boxes, 300, 23, cp, H, ft)
    for v in range(y.shape[0]):
        mom, pr = ora.summarize_set(rb["accept_idx"][v], models, boxes, 300, 23, bank_theta=th_b)
        assert np.allclose(mom, rb["moments"][v], rtol=1e-12, atol=1e-15, equal_nan=True)
        assert np.array_equal(pr, rb["model_prob"][v])
    # a set of IRR draws only: probability 1 for IRR, the plain mean of those draws
    idx = np.arange(300, 320)
    mom, pr = ora.summarize_set(idx, models, boxes, 300, 23, bank_theta=th_b)
    assert np.array_equal(pr, [0.0, 1.0, 0.0])
    assert np.allclose(mom[1, 0, 0], th_b[idx, 0].astype(np.float64).mean(), rtol=1e-14)
    assert np.isnan(mom[0]).all() and np.isnan(mom[2]).all()
