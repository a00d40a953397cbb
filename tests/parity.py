"""Comparison helpers for GPU-vs-oracle parity (the tolerances of the hot path).

  * draws: Philox words and fp32 theta bit-identical;
  * TACs: max_f |x_gpu - x_ora| <= 1e-5 * max_f |x_ora| per row;
  * accepted sets: identical except draws whose oracle distance lies within
    1e-5 (relative) of the oracle's threshold;
  * posterior means within 1e-3 relative (checked tighter where the sets agree:
    both sides reduce in FP64, so only the fp32 output rounding differs).
"""
import numpy as np

import workloads as W

TAC_RTOL = 1e-5
THRESH_RTOL = 1e-5
MEAN_RTOL = 1e-3


def tac_rel_err(gpu, ora):
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    return np.abs(gpu - ora).max(axis=1) / np.abs(ora).max(axis=1)


def compare_sets(ora_mod, gpu_idx, ora_res, y, ft, cp, dt, models, boxes, n_draws, seed, voxel_offset=0,
                 l1=False, weights=None):
    """Returns (n_voxels_with_swaps, list of (v, g, rel_gap)) and asserts the swap rule."""
    swaps = []
    nvox = 0
    for v in range(gpu_idx.shape[0]):
        a_g, a_o = set(gpu_idx[v].tolist()), set(ora_res["accept_idx"][v].tolist())
        if a_g == a_o:
            continue
        nvox += 1
        h = ora_res["threshold"][v]
        d = ora_mod.voxel_distances(y[v], ft, cp, dt, models, boxes, n_draws, seed, v + voxel_offset, l1=l1,
                                    weights_v=None if weights is None else weights[v])
        for g in a_g ^ a_o:
            gap = abs(d[g] - h) / h
            swaps.append((v, g, gap))
            assert gap <= THRESH_RTOL, f"voxel {v}: draw {g} swapped at relative gap {gap:.3e} from the threshold"
    return nvox, swaps


def oracle_moments_of(ora_mod, models, boxes, seed, v_global, idx, n_draws):
    """FP64 moments of an explicit accepted set (the oracle's reduction rule)."""
    M = len(models)
    n = len(idx)
    idx = np.asarray(idx, dtype=np.int64)
    m = idx // n_draws
    i = idx % n_draws
    _, _, th = ora_mod.draws(models, boxes, seed, np.full(n, v_global), i, m)
    t = th.astype(np.float64)
    t[:, 5] = t[:, 0] * t[:, 2] / (t[:, 1] + t[:, 2])
    mom = np.full((M, 8, 2), np.nan)
    prob = np.zeros(M)
    for mm in range(M):
        sel = t[m == mm]
        prob[mm] = sel.shape[0] / n
        if sel.shape[0] == 0:
            continue
        mom[mm, :, 0] = sel.mean(axis=0)
        mom[mm, :, 1] = sel.var(axis=0, ddof=1) if sel.shape[0] > 1 else 0.0
        if models[mm] == 1:
            mom[mm, [2, 3, 5]] = np.nan
        elif models[mm] == 2:
            mom[mm, 3] = np.nan
        mom[mm, 6:] = np.nan
    return mom, prob


def spread_sample(n_voxels, k=40, seed=0, edges=(256, 131072, 262144)):
    """Sorted, unique voxel indices spread over a volume: the first and last two
    voxels, both sides of the first few multiples of every size in `edges`
    (workgroup blocks and voxel chunks of the launches) and of the last one,
    the rest uniform at random; at least k of them."""
    s = {0, 1, n_voxels - 2, n_voxels - 1}
    for e in edges:
        mults = list(range(e, n_voxels, e))
        for b in mults[:2] + mults[-1:]:
            s.update((b - 1, b))
    rng = np.random.default_rng(seed)
    while len(s) < k:
        s.add(int(rng.integers(0, n_voxels)))
    return np.array(sorted(v for v in s if 0 <= v < n_voxels), dtype=np.int64)


_VOLUMES = {}


def large_volume(cfg):
    """Observed TACs of every voxel of the 1M-voxel irreversible-2TCM
    configuration: oracle curves of the seeded true parameters plus the seeded
    noise (each voxel its own curve; cached per process)."""
    import oracle as ora
    if cfg.name not in _VOLUMES:
        th, eps = cfg.truth()
        clean = ora.simulate(cfg.models[0], th, cfg.input_fn(), cfg.dt, cfg.frame_times)
        _VOLUMES[cfg.name] = (th, W.add_noise(clean, cfg.frame_times, eps))
    return _VOLUMES[cfg.name]


def check_voxels(g_idx, g_mom, g_prob, o, dist_of, moments_of, mean_rtol=1e-5, var_rtol=1e-4, mean_atol=1e-7,
                 var_atol=1e-9, prob_atol=1e-7, label=""):
    """Every row j (a sampled voxel): the GPU's accepted set equals the
    oracle's except draws whose oracle distance lies within THRESH_RTOL of
    the oracle's threshold (dist_of(j): oracle distances of every draw, by
    global index); the moments and model probabilities equal the oracle's
    (its outputs when the sets agree, its FP64 reduction of the GPU's own set,
    moments_of(j, idx) -> (mom, prob), when they differ).  No voxel is
    exempt.  Returns the number of voxels with threshold swaps."""
    swaps = 0
    for j in range(g_idx.shape[0]):
        gi = np.asarray(g_idx[j])
        a_g, a_o = set(gi.tolist()), set(np.asarray(o["accept_idx"][j]).tolist())
        assert len(a_g) == gi.size, f"{label} row {j}: repeated draw indices"
        if a_g == a_o:
            ref_mom, ref_prob = o["moments"][j], o["model_prob"][j]
        else:
            swaps += 1
            d = dist_of(j)
            h = o["threshold"][j]
            for g in a_g ^ a_o:
                gap = abs(d[g] - h) / h
                assert gap <= THRESH_RTOL, f"{label} row {j}: draw {g} swapped at relative gap {gap:.3e}"
            ref_mom, ref_prob = moments_of(j, gi)
        gm = np.asarray(g_mom[j], dtype=np.float64)
        assert np.array_equal(np.isnan(gm), np.isnan(ref_mom)), f"{label} row {j}: NaN pattern"
        ok = ~np.isnan(ref_mom)
        assert np.allclose(gm[..., 0][ok[..., 0]], ref_mom[..., 0][ok[..., 0]], rtol=mean_rtol, atol=mean_atol), \
            f"{label} row {j}: means"
        assert np.allclose(gm[..., 1][ok[..., 1]], ref_mom[..., 1][ok[..., 1]], rtol=var_rtol, atol=var_atol), \
            f"{label} row {j}: variances"
        assert np.allclose(np.asarray(g_prob[j], dtype=np.float64), ref_prob, rtol=0, atol=prob_atol,
                           equal_nan=True), f"{label} row {j}: model probabilities"
    return swaps


def bank_distances(ora_mod, y_v, x_bank, ft, dt, n_nodes, l1=False, weights_v=None, lam=None):
    """Oracle distances of one voxel to every bank row (FP64, the pinned weights)."""
    kw = {} if lam is None else {"lam": lam}
    w = ora_mod.weights(y_v, ft, dt, n_nodes, **kw) if weights_v is None else np.asarray(weights_v, np.float64)
    r = np.asarray(y_v, dtype=np.float64) - x_bank
    return (np.sqrt(w) * np.abs(r)).sum(1) if l1 else (w * r * r).sum(1)
