"""Pins for the oracle of the shared bank drawn from a learned proposal (not in
the paper; definitions in oracle/learned_bank.py).

  * the serpentine cell numbering is a bijection onto 0 .. bins^D - 1 whose
    consecutive numbers are neighbouring cells (brute force over every grid);
  * a voxel's mixture mean and second moment are those of draws from the
    mixture (the sampler of oracle/proposal.py, an independent route);
  * the group Gaussian of members that share one mixture is that mixture's
    mean and variance;
  * bank rows: the Gaussian part has the group's mean and sd in z; a prior
    share of 1 draws the prior box with unit weights; and, with every row
    counted, the importance-weighted parameter means are the prior means
    (pins the draws, the Jacobian term, the box widths and the defensive
    mixture together) for both models and both heads;
  * end to end: at plain ABC's own threshold the learned bank's weighted
    Ki mean agrees with plain ABC's (the same ABC target, Eq. (7)), and two
    identical models (k4 fixed at 0) share the probability evenly.
"""
import itertools
import math

import numpy as np

import oracle as ora
import oracle.learned_bank as lb
import oracle.proposal as prop
import workloads as W

IRR, REV = W.M_2TCM_IRR, W.M_2TCM_REV


def test_serpentine_cells_are_a_walk_through_neighbours():
    for bins, D in ((1, 4), (2, 3), (3, 4), (4, 5), (8, 4), (5, 5)):
        lo, wid = np.zeros(D), np.ones(D)
        cells = np.array(list(itertools.product(range(bins), repeat=D)))
        m = np.log((cells + 0.5) / bins)  # exp(m) at the cell centres
        key = lb.cell_keys(m, bins, lo, wid)
        assert np.array_equal(np.sort(key), np.arange(bins ** D))
        walk = cells[np.argsort(key)]
        steps = np.abs(np.diff(walk, axis=0))
        assert np.all(steps.sum(axis=1) == 1), (bins, D)
    # clamping: below the box -> 0, above -> bins - 1
    key = lb.cell_keys(np.log(np.array([[1e-9, 1e-9], [50.0, 50.0]])), 3, np.array([0.1, 0.1]), np.array([1.0, 1.0]))
    assert key[0] == 0 and key[1] == lb.cell_keys(np.log(np.array([[1.05, 1.05]])), 3, np.full(2, 0.1), np.ones(2))[0]


def _outputs(rng, n, dims, centre, spread=0.3, sd=0.3):
    o = np.zeros((n, 96))
    o[:, :prop.C] = rng.standard_normal((n, prop.C))
    o[:, prop.C:prop.C + prop.C * dims] = (np.repeat(centre[:, None, :], prop.C, axis=1)
                                           + spread * rng.standard_normal((n, prop.C, dims))).reshape(n, -1)
    s = (math.log(sd) - prop.LS0) / (prop.LS1 - prop.LS0)
    o[:, prop.C + prop.C * dims:prop.C + 2 * prop.C * dims] = (math.log(s / (1 - s))
                                                               + 0.3 * rng.standard_normal((n, prop.C * dims)))
    return o


def test_mixture_moments_match_draws_from_the_mixture(ora):
    rng = np.random.default_rng(1)
    o = _outputs(rng, 1, 4, np.array([[-1.0, -1.5, -2.0, -3.0]]))
    m, s = lb.summaries(o, 4)
    z, _ = prop.draws(o[0, :prop.NOUT], prop.philox_words(5, 300_000, 3))
    se = np.sqrt((s[0] - m[0] ** 2) / z.shape[0])
    assert np.all(np.abs(z.mean(axis=0) - m[0]) < 4.5 * se)
    assert np.allclose((z * z).mean(axis=0), s[0], rtol=0.02)


def test_group_gaussian_of_identical_members_is_the_mixture():
    rng = np.random.default_rng(2)
    V = 300
    o1 = _outputs(rng, 1, 5, np.array([[-1.0, -1.0, -2.0, -3.5, -3.0]]))
    o = np.repeat(o1, V, axis=0)
    y = np.ones((V, 30), dtype=np.float32)
    box = W.box_array([REV])[0]
    key, order, group, mu, sd, cnt = lb.grouping(y, o, 5, 2, 256, box, 1.5)
    m, s = lb.summaries(o1, 5)
    assert cnt.tolist() == [256, 44] and np.all(key == key[0])
    assert np.array_equal(order, np.arange(V))  # ties keep voxel order
    for g in range(2):
        assert np.allclose(mu[g], m[0].astype(np.float32), rtol=1e-6)
        assert np.allclose(sd[g], (np.sqrt(s[0] - m[0] ** 2) * 1.5).astype(np.float32), rtol=1e-6)
    y[3, 2] = np.nan  # an invalid voxel sorts last and leaves the fit
    key, order, group, mu2, sd2, cnt = lb.grouping(y, o, 5, 2, 256, box, 1.5)
    assert order[-1] == 3 and group[3] == 1 and cnt.tolist() == [256, 43]


def _rows(models, dims, share, n, mu=None, sd=None, seed=11):
    boxes = W.box_array(models)
    mu = np.array([-0.7, -1.0, -2.2, -3.3, -3.3] if dims == 5 else [-0.7, -1.0, -2.2, -3.3]) if mu is None else mu
    sd = np.full(dims, 0.25) if sd is None else sd
    th, lw, ok = lb.bank_rows(7, mu, sd, 1, models, boxes, dims, n, share, seed)
    return boxes, mu, sd, th, lw, ok


def test_gaussian_part_of_the_rows_has_the_group_moments(ora):
    for models, dims in (([IRR], 4), ([REV], 5)):
        boxes, mu, sd, th, lw, ok = _rows(models, dims, 0.0, 200_000)
        slots = lb.MODEL_SLOTS[models[0]]
        z = np.log(th[:, list(slots)].astype(np.float64))
        assert ok.mean() > 0.99  # the Gaussians sit well inside the box
        zz = z[ok]
        se = sd / math.sqrt(zz.shape[0])
        assert np.all(np.abs(zz.mean(axis=0) - mu) < 4.5 * se + 1e-7), (zz.mean(axis=0), mu)
        assert np.allclose(zz.std(axis=0), sd, rtol=0.02)


def test_prior_share_one_draws_the_box_with_unit_weights(ora):
    boxes, _, _, th, lw, ok = _rows([IRR, REV], 4, 1.0, 100_000)
    assert ok.all() and np.all(lw == 0.0)
    for mi, model in enumerate([IRR, REV]):
        rows = th[mi * 100_000:(mi + 1) * 100_000]
        for s in lb.MODEL_SLOTS[model]:
            lo, hi = boxes[mi][s]
            t = rows[:, s].astype(np.float64)
            assert t.min() >= np.float32(lo) and t.max() <= np.float32(hi)
            assert abs(t.mean() - 0.5 * (lo + hi)) < 4.5 * (hi - lo) / math.sqrt(12 * t.size)


def test_weighted_rows_recover_the_prior_means(ora):
    """Every row counted: sum w theta / sum w -> the box midpoint, for both
    models under a four- and a five-parameter head (k4 from u_6 or from the
    head), while the unweighted means of the same rows miss."""
    for dims in (4, 5):
        mu = np.array([-0.9, -1.2, -2.0, -3.0, -2.6])[:dims] if dims == 5 else np.array([-0.9, -1.2, -2.0, -2.6])
        boxes, mu, sd, th, lw, ok = _rows([IRR, REV], dims, 0.2, 300_000, mu=mu, sd=np.full(dims, 0.9))
        for mi, model in enumerate([IRR, REV]):
            r = slice(mi * 300_000, (mi + 1) * 300_000)
            w = np.exp(lw[r] - lw[r][ok[r]].max()) * ok[r]
            ess = w.sum() ** 2 / (w * w).sum()
            missed = False
            for s in lb.MODEL_SLOTS[model]:
                lo, hi = boxes[mi][s]
                t = np.nan_to_num(th[r, s].astype(np.float64))
                est = (w * t).sum() / w.sum()
                se = (hi - lo) / math.sqrt(12 * ess)
                assert abs(est - 0.5 * (lo + hi)) < 4.5 * se, (dims, model, s, est, se)
                missed |= abs(t[ok[r]].mean() - 0.5 * (lo + hi)) > 10 * se
            assert missed


def _voxels(n, seed, model=IRR):
    cfg = W.CFG_LARGE
    ft, cp = cfg.frame_times, cfg.input_fn()
    rng = np.random.default_rng(seed)
    th = W.true_params(rng, n, model, W.box_array([model])[0])
    y = W.add_noise(ora.simulate(model, th, cp, cfg.dt, ft), ft, rng.standard_normal((n, ft.size - 1)))
    return cfg, ft, cp, th, y, rng


def test_learned_bank_at_plain_threshold_matches_plain_abc(ora):
    """256 voxels with nearby truths in one group, a 40k-row bank from the
    group's proposal; restricted to plain ABC's own threshold (400k prior
    draws, 400 accepted) the weighted Ki mean agrees with plain ABC's within
    Monte Carlo error."""
    cfg, ft, cp, th, y, rng = _voxels(256, 21)
    th[:] = th[0]
    th[:, list(prop.FREE_SLOTS)] *= np.exp(0.05 * rng.standard_normal((256, 4)))
    y = W.add_noise(ora.simulate(IRR, th, cp, cfg.dt, ft), ft, rng.standard_normal(y.shape))
    centre = np.log(np.maximum(th[:, list(prop.FREE_SLOTS)], 1e-3))
    o = _outputs(rng, 256, 4, centre, spread=0.1, sd=0.25)
    box = W.box_array([IRR])
    vox = [0, 1, 2]
    below = np.full(256, np.nan, dtype=np.float32)
    ref = {}
    for v in vox:
        r = ora.infer(y[v:v + 1], ft, cp, cfg.dt, [IRR], box, 400_000, 0.001, 5, voxel_offset=v)
        below[v] = np.float32(r["threshold"][0])
        ref[v] = r["moments"][0, 0, 5]
    out = lb.infer_bank_learned(y, ft, cp, cfg.dt, [IRR], box, o, 40_000, 0.05, 9, dims=4, bins=1,
                                group_voxels=256, prior_share=0.2, sd_scale=1.5, accept_below=below, voxels=vox)
    for k, v in enumerate(vox):
        assert out["threshold"][k] > below[v]  # every row at or below h_v was kept
        mean, var = out["moments"][k, 0, 5]
        se = math.sqrt(var / out["ess"][k] + ref[v][1] / 400.0)
        print(f"voxel {v}: Ki plain {ref[v][0]:.5f} learned bank {mean:.5f} (SE {se:.1e}, ESS {out['ess'][k]:.0f})")
        assert out["ess"][k] > 20 and abs(mean - ref[v][0]) <= 4.0 * se


def test_identical_models_share_the_probability(ora):
    """IRR and REV with k4 fixed at 0 are the same model: over 256 voxels the
    weighted probability of the second is 0.5 within Monte Carlo error."""
    cfg, ft, cp, th, y, rng = _voxels(256, 22)
    centre = np.log(np.maximum(th[:, list(prop.FREE_SLOTS)], 1e-3))
    o = _outputs(rng, 256, 4, centre, spread=0.2, sd=0.3)
    boxes = W.box_array([IRR, REV])
    boxes[1][3] = (0.0, 0.0)
    out = lb.infer_bank_learned(y, ft, cp, cfg.dt, [IRR, REV], boxes, o, 4000, 0.01, 13, dims=4, bins=2,
                                group_voxels=256, prior_share=0.2, voxels=np.arange(0, 256, 8))
    p = out["model_prob"][:, 1]
    se = math.sqrt(0.25 / np.nanmean(out["ess"]) / p.size)
    assert abs(np.nanmean(p) - 0.5) < 4.5 * se, (np.nanmean(p), se)
    assert np.allclose(out["model_prob"].sum(axis=1), 1.0)
