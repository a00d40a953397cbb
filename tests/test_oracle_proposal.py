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
