"""Pins for the oracle of the learned proposal and importance-weighted ABC
(not in the paper; see oracle/proposal.py for the definitions).

  * every gradient agrees with central finite differences (FP64);
  * the mixture log density agrees with a direct sum of scipy normal densities;
  * draws from the mixture have its analytic mean and variance;
  * with every draw accepted, the importance-weighted means of the parameters
    are the prior (box) means: this pins the weight, its Jacobian term and the
    sampler together;
  * Adam's first step is lr * sign(g); training lowers the loss.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle.proposal as prop
import workloads as W


def _tiny_params(rng):
    return prop.init_params(rng)


def test_gradients_match_finite_differences(ora):
    rng = np.random.default_rng(0)
    p = _tiny_params(rng)
    for k in p:  # non-zero biases so that every path is exercised
        if k.startswith("b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = prop.features(np.abs(rng.standard_normal((6, 30))) * 5.0)
    z = rng.standard_normal((6, prop.D)) - 1.0
    _, g = prop.loss_and_grad(p, x, z)
    for k, shape in ((k, p[k].shape) for k in p):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in shape)
            if k == "W1" and idx[0] >= 30:
                continue  # padded inputs are always 0
            old = p[k][idx]
            h = 1e-6 * max(1.0, abs(old))
            p[k][idx] = old + h
            lp, _ = prop.loss_and_grad(p, x, z)
            p[k][idx] = old - h
            lm, _ = prop.loss_and_grad(p, x, z)
            p[k][idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_log_density_against_direct_sum():
    rng = np.random.default_rng(1)
    o = rng.standard_normal((5, prop.NOUT))
    logpi, mu, logsd = prop.mixture(o)
    z = mu[:, 0, :] + 0.5 * rng.standard_normal((5, prop.D))  # where the density does not underflow
    for b in range(5):
        dens = 0.0
        for c in range(prop.C):
            dens += math.exp(logpi[b, c]) * np.prod(stats.norm.pdf(z[b], loc=mu[b, c], scale=np.exp(logsd[b, c])))
        assert prop.log_density(o[b:b + 1], z[b:b + 1])[0] == pytest.approx(math.log(dens), rel=1e-10, abs=1e-10)
    assert np.all(logsd >= prop.LS0) and np.all(logsd <= prop.LS1)


def test_draws_have_the_mixture_moments(ora):
    rng = np.random.default_rng(2)
    o = rng.standard_normal(prop.NOUT)
    words = prop.philox_words(17, 200_000, 9)
    z, th = prop.draws(o, words)
    logpi, mu, logsd = prop.mixture(o[None, :])
    pi, mu, sd = np.exp(logpi[0]), mu[0], np.exp(logsd[0])
    mean = (pi[:, None] * mu).sum(axis=0)
    var = (pi[:, None] * (sd ** 2 + mu ** 2)).sum(axis=0) - mean ** 2
    se = np.sqrt(var / z.shape[0])
    assert np.all(np.abs(z.mean(axis=0) - mean) < 4.5 * se)
    assert np.allclose(z.var(axis=0), var, rtol=0.02)
    assert np.array_equal(th, np.exp(z).astype(np.float32))


def test_importance_weights_recover_the_prior_means(ora):
    """All draws accepted: sum w theta / sum w -> E_prior[theta] = box midpoint."""
    rng = np.random.default_rng(3)
    box = W.box_array([W.M_2TCM_IRR])[0]
    lo = np.array([box[s][0] for s in prop.FREE_SLOTS])
    hi = np.array([box[s][1] for s in prop.FREE_SLOTS])
    # a broad proposal that covers the box: two components around its log-centre
    o = np.zeros(prop.NOUT)
    mu = np.log(np.sqrt(np.maximum(lo, 1e-3) * hi))
    o[prop.C:prop.C + prop.C * prop.D] = np.tile(mu, prop.C) + 0.3 * rng.standard_normal(prop.C * prop.D)
    o[prop.C + prop.C * prop.D:] = 1.5  # sd ~ e^{0.6}
    words = prop.philox_words(3, 400_000, 21)
    z, th = prop.draws(o, words)
    valid = np.all((th >= lo.astype(np.float32)) & (th <= hi.astype(np.float32)), axis=1)
    lw = prop.log_weight(o, z[valid])
    w = np.exp(lw - lw.max())
    t = th[valid].astype(np.float64)
    est = (w[:, None] * t).sum(axis=0) / w.sum()
    ess = w.sum() ** 2 / (w * w).sum()
    se = np.sqrt((hi - lo) ** 2 / 12.0 / ess)
    assert np.all(np.abs(est - 0.5 * (lo + hi)) < 4.5 * se), (est, 0.5 * (lo + hi), se)
    # and the same draws weighted 1 are far from it (the check has power)
    assert np.any(np.abs(t.mean(axis=0) - 0.5 * (lo + hi)) > 10 * se)


def test_adam_first_step_and_training_lowers_loss():
    p = {"a": np.array([1.0, -2.0])}
    st = {}
    prop.adam(p, {"a": np.array([0.3, -5.0])}, st, lr=0.01)
    assert np.allclose(p["a"], [1.0 - 0.01, -2.0 + 0.01], atol=1e-9)
    rng = np.random.default_rng(4)
    q = prop.init_params(rng)
    x = prop.features(np.abs(rng.standard_normal((256, 30))) * 3.0)
    z = 0.5 * x[:, :prop.D] - 1.0 + 0.1 * rng.standard_normal((256, prop.D))
    l0, _ = prop.loss_and_grad(q, x, z)
    st = {}
    for _ in range(150):
        _, g = prop.loss_and_grad(q, x, z)
        prop.adam(q, g, st, lr=1e-3)
    l1, _ = prop.loss_and_grad(q, x, z)
    assert l1 < l0 - 1.0, (l0, l1)


def _box():
    box = W.box_array([W.M_2TCM_IRR])[0]
    lo = np.array([np.float32(box[s][0]) for s in prop.FREE_SLOTS], dtype=np.float64)
    hi = np.array([np.float32(box[s][1]) for s in prop.FREE_SLOTS], dtype=np.float64)
    return lo, hi


def test_defensive_share_draws_the_prior_and_keeps_the_target(ora):
    """Defensive mixture a p + (1 - a) q: a share 1 gives uniform draws on the
    box with equal weights; a share 0.3 draws that fraction from the prior and,
    with every draw accepted, the weighted means are still the prior means."""
    lo, hi = _box()
    rng = np.random.default_rng(5)
    o = rng.standard_normal(prop.NOUT)
    words = prop.philox_words(11, 100_000, 4)
    z, th = prop.draws(o, words, lo, hi, prior_share=1.0)
    assert np.all((th >= lo.astype(np.float32)) & (th <= hi.astype(np.float32)))
    assert np.allclose(th.mean(axis=0), 0.5 * (lo + hi), atol=4.5 * np.sqrt((hi - lo) ** 2 / 12 / 1e5))
    lw = prop.log_weight(o, z, lo, hi, prior_share=1.0)
    assert np.all(lw == 0.0)
    # a share of 0.3 around a broad proposal
    o = np.zeros(prop.NOUT)
    o[prop.C:prop.C + prop.C * prop.D] = np.tile(np.log(np.sqrt(np.maximum(lo, 1e-3) * hi)), prop.C)
    o[prop.C + prop.C * prop.D:] = 1.0
    words = prop.philox_words(3, 400_000, 22)
    z, th = prop.draws(o, words, lo, hi, prior_share=0.3)
    w = words.astype(np.uint64)
    u0 = ((w[:, 0] & 255) | (w[:, 1] & 255) << 8 | (w[:, 2] & 255) << 16) * 2.0 ** -24
    frac = np.mean(u0 < 0.3)
    assert abs(frac - 0.3) < 4.5 * math.sqrt(0.3 * 0.7 / words.shape[0])
    valid = np.all((th >= lo.astype(np.float32)) & (th <= hi.astype(np.float32)), axis=1)
    lw = prop.log_weight(o, z[valid], lo, hi, prior_share=0.3)
    assert np.all(lw <= -math.log(0.3) + 1e-12)  # every weight below 1 / a
    w = np.exp(lw - lw.max())
    est = (w[:, None] * th[valid].astype(np.float64)).sum(axis=0) / w.sum()
    ess = w.sum() ** 2 / (w * w).sum()
    se = np.sqrt((hi - lo) ** 2 / 12.0 / ess)
    assert np.all(np.abs(est - 0.5 * (lo + hi)) < 4.5 * se), (est, se)
    # the same draws weighted as if the share were 0 miss (the share term matters)
    lw0 = prop.log_weight(o, z[valid], lo, hi, prior_share=0.0)
    w0 = np.exp(lw0 - lw0.max())
    est0 = (w0[:, None] * th[valid].astype(np.float64)).sum(axis=0) / w0.sum()
    assert np.any(np.abs(est0 - 0.5 * (lo + hi)) > 10 * se)


def test_sd_scale_widens_every_component():
    rng = np.random.default_rng(6)
    o = rng.standard_normal(prop.NOUT)
    o[:prop.C] = -50.0
    o[0] = 50.0  # one component
    words = prop.philox_words(2, 200_000, 8)
    z1, _ = prop.draws(o, words)
    z2, _ = prop.draws(o, words, sd_scale=2.5)
    logpi, mu, logsd = prop.mixture(o[None, :])
    assert np.allclose(z2 - mu[0, 0], 2.5 * (z1 - mu[0, 0]), rtol=1e-12, atol=1e-12)
    sd = np.exp(logsd[0, 0]) * 2.5
    lq = prop.log_density(o[None, :], z2[:1], sd_scale=2.5)[0]
    assert lq == pytest.approx(np.sum(stats.norm.logpdf(z2[0], loc=mu[0, 0], scale=sd)), rel=1e-9, abs=1e-9)


def _is_setup(nv, seed):
    import oracle as ora
    cfg = W.CFG_LARGE
    ft, cp = cfg.frame_times, cfg.input_fn()
    box = W.box_array([W.M_2TCM_IRR])
    rng = np.random.default_rng(seed)
    th = W.true_params(rng, nv, W.M_2TCM_IRR, box[0])
    y = W.add_noise(ora.simulate(W.M_2TCM_IRR, th, cp, cfg.dt, ft), ft, rng.standard_normal((nv, ft.size - 1)))
    return cfg, ft, cp, box, th, y, rng


def _centred_outputs(th_v, rng, sd=0.4):
    o = np.zeros(prop.NOUT)
    z0 = np.log(np.maximum(th_v[list(prop.FREE_SLOTS)], 1e-3))
    o[prop.C:prop.C + prop.C * prop.D] = np.tile(z0, prop.C) + 0.2 * rng.standard_normal(prop.C * prop.D)
    s = (math.log(sd) - prop.LS0) / (prop.LS1 - prop.LS0)
    o[prop.C + prop.C * prop.D:] = math.log(s / (1.0 - s))
    return o


def test_given_threshold_is_the_prefix_of_the_fixed_fraction(ora):
    """ABC at a given threshold h (the indicator form of Eq. (7)) keeps, of the
    n closest draws, those at or below h.  With h the k-th smallest distance
    (k < n) that is exactly the fixed-fraction result with k accepted draws;
    with h = inf it is the fixed-fraction result itself."""
    cfg, ft, cp, box, th, y, rng = _is_setup(3, 41)
    for v in range(3):
        o = _centred_outputs(th[v], rng)
        kw = dict(prior_share=0.2, sd_scale=1.3)
        order, mom, ess, d = prop.infer_is(y[v], ft, cp, cfg.dt, box[0], o, 4000, 0.05, 7, v, **kw)
        k = 37
        h = np.float32(d[order[k - 1]])
        assert np.float32(d[order[k]]) > h  # distinct at the cut
        _, mom_h, ess_h, _ = prop.infer_is(y[v], ft, cp, cfg.dt, box[0], o, 4000, 0.05, 7, v, accept_below=h, **kw)
        _, mom_k, ess_k, _ = prop.infer_is(y[v], ft, cp, cfg.dt, box[0], o, 4000, k / 4000, 7, v, **kw)
        assert np.array_equal(mom_h, mom_k, equal_nan=True) and ess_h == ess_k
        _, mom_inf, ess_inf, _ = prop.infer_is(y[v], ft, cp, cfg.dt, box[0], o, 4000, 0.05, 7, v,
                                               accept_below=np.float32(np.inf), **kw)
        assert np.array_equal(mom_inf, mom, equal_nan=True) and ess_inf == ess
        _, mom_0, ess_0, _ = prop.infer_is(y[v], ft, cp, cfg.dt, box[0], o, 4000, 0.05, 7, v,
                                           accept_below=np.float32(0.5 * d[order[0]]), **kw)
        assert np.isnan(mom_0).all() and np.isnan(ess_0)


def test_importance_weighted_abc_at_plain_threshold_matches_plain_abc(ora):
    """Plain prior ABC (Alg. 1) with 400k draws, 400 accepted, sets a threshold
    h; importance-weighted ABC with 40k draws from a proposal centred near the
    truth, restricted to the same h, targets the same distribution (the prior
    on {d <= h}), so its weighted Ki mean agrees with plain ABC's within
    Monte Carlo error.  Weighting the same draws by 1 instead misses (the
    proposal favours the middle of the region)."""
    cfg, ft, cp, box, th, y, rng = _is_setup(3, 42)
    n_pl, p_pl, n_is, p_is = 400_000, 0.001, 100_000, 0.039
    for v in range(3):
        ref = ora.infer(y[v:v + 1], ft, cp, cfg.dt, [W.M_2TCM_IRR], box, n_pl, p_pl, 5, voxel_offset=v)
        h = np.float32(ref["threshold"][0])
        ki_pl, var_pl = ref["moments"][0, 0, 5]
        o = _centred_outputs(th[v], rng, sd=0.3)
        order, mom, ess, d = prop.infer_is(y[v], ft, cp, cfg.dt, box[0], o, n_is, p_is, 9, v, prior_share=0.1,
                                           sd_scale=1.0, accept_below=h)
        assert np.float32(d[order[-1]]) > h  # every draw below h was kept
        ki_is, var_is = mom[5]
        se = math.sqrt(var_is / ess + var_pl / 400.0)
        print(f"voxel {v}: Ki plain {ki_pl:.5f} IS {ki_is:.5f} (SE {se:.2e}, ESS {ess:.0f})")
        assert ess > 20 and abs(ki_is - ki_pl) <= 4.0 * se
