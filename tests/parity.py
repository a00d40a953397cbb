"""Comparison helpers for GPU-vs-oracle parity (the tolerances of the hot path).

  * draws: Philox words and fp32 theta bit-identical;
  * TACs: max_f |x_gpu - x_ora| <= 1e-5 * max_f |x_ora| per row;
  * accepted sets: identical except draws whose oracle distance lies within
    1e-5 (relative) of the oracle's threshold;
  * posterior means within 1e-3 relative (checked tighter where the sets agree:
    both sides reduce in FP64, so only the fp32 output rounding differs).
"""
import numpy as np

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
