"""FP64 oracle of the shared bank drawn from a learned proposal.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain numpy and the C
oracle's forward model, FP64, written from the definitions below; it shares no
code with the GPU library.

Not in the paper.  Alg. 1 simulates one bank of prior draws and scores every
voxel against it (lines 1-4).  Here the bank is drawn from a proposal instead
of the prior, one bank per group of voxels, and each bank row carries the
importance weight prior / proposal, so that each voxel's ABC target (the prior
restricted to {d <= h}, Eq. (7)) is unchanged.  Definitions, in the order the
method applies them:

1. voxel summary: the network's mixture for voxel v (a head over D = dims
   parameters, see ``oracle.proposal``) has, per parameter j, mean
   m_j = sum_c pi_c mu_cj and second moment s_j = sum_c pi_c (sd_cj^2 + mu_cj^2);
2. cell: coordinate b_j = floor(bins (exp(m_j) - lo_j) / wid_j) clamped to
   [0, bins - 1] (lo_j, wid_j = hi_j - lo_j of the prior box in fp32), and the
   cells are numbered along a serpentine walk: key = 0; for each j in order,
   c = b_j, reversed (bins - 1 - b_j) when key is odd, key = key * bins + c.
   An invalid voxel (a non-finite or negative caller weight, a non-finite
   observation, max_f y <= 0, or a non-finite mixture moment) gets key
   bins^D;
3. groups: voxels sorted by key, ties by voxel index; position p belongs to
   group p // S;
4. group Gaussian: over the group's valid members, mu_j = mean of m_j and
   var_j = mean of s_j - mu_j^2 (at least 1e-12), sd_j = sqrt(var_j) * scale;
   both rounded to fp32.  No valid member: the group's rows are prior draws
   with weight 1;
5. bank rows: row i of model position m of group g takes Philox4x32-10 words
   w = philox(i, G0 + g, 3, m << 16) and v = philox(i, G0 + g, 3, m << 16 | 1)
   (key = seed; G0 a given first group number, 0 by default); u0 = ((w0 & 255) | (w1 & 255) << 8 | (w2 & 255) << 16) 2^-24,
   u_p = (w_p >> 8) 2^-24 (p < 4), u_4, u_5, u_6 = (v_0, v_1, v_2 >> 8) 2^-24.
   If u0 < a (or the group is empty) every parameter is uniform,
   theta_p = fp32(lo_p + u_p wid_p); otherwise a parameter with a head
   parameter d is theta_p = fp32(exp(z_p)), z_p = mu_d + sd_d n_p with the
   Box-Muller normals n_2q, n_2q+1 = r cos(2 pi u_2q+1), r sin(2 pi u_2q+1),
   r = sqrt(-2 ln(u_2q + 2^-24)) (invalid outside [lo_p, lo_p + wid_p]), and
   a parameter without one (k4 under a four-parameter head) is
   fp32(lo_p + u_6 wid_p).  A parameter whose box has zero width is lo_p;
6. weight: L = sum over parameters with a head parameter and a box of
   non-zero width of [log N(z_p; mu_d, sd_d) - z_p + log wid_p] (z_p = log
   theta_p for a uniform draw); log w = -log(a + (1 - a) e^L), with L = -inf
   (a parameter at 0) giving w = 1 / a; an invalid row has log w = -inf and
   no curve;
7. each voxel: the fixed-budget selection of the plain method against its
   group's bank rows (distance sum_f w_f (y_f - x_f)^2 or sum_f sqrt(w_f)
   |y_f - x_f|, keys (fp32(d), row) with an undefined distance last); the
   n = floor(M n_draws p + 1e-6) smallest kept; those at or below a given
   threshold (if any) count with their weights: probability of model m =
   sum_m w / sum w, weighted mean and variance sum w (t - mean)^2 / sum w of
   each parameter and of Ki = K1 k3 / (k2 + k3), ESS = (sum w)^2 / sum w^2.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as ora
import oracle.proposal as prop

HEAD_SLOTS = {4: (0, 1, 2, 4), 5: (0, 1, 2, 3, 4)}
MODEL_SLOTS = {ora.M_2TCM_IRR: (0, 1, 2, 4), ora.M_2TCM_REV: (0, 1, 2, 3, 4)}


def summaries(o, dims):
    """Per voxel mixture mean m [V][D] and second moment s [V][D] of z."""
    logpi, mu, logsd = prop.mixture(np.asarray(o, dtype=np.float64), dims=dims)
    pi = np.exp(logpi)[:, :, None]
    return (pi * mu).sum(axis=1), (pi * (np.exp(2.0 * logsd) + mu * mu)).sum(axis=1)


def box32(box_m, slots):
    """fp32 lo and fp32 width (hi - lo rounded once) of the given slots."""
    lo = np.array([np.float32(box_m[s][0]) for s in slots], dtype=np.float64)
    wid = np.array([np.float32(box_m[s][1] - box_m[s][0]) for s in slots], dtype=np.float64)
    return lo, wid


def cell_keys(m, bins, lo, wid):
    """Serpentine cell number of each voxel from its mixture means m [V][D]."""
    wid = np.where(wid > 0.0, wid, 1.0)
    key = np.zeros(m.shape[0], dtype=np.int64)
    for j in range(m.shape[1]):
        b = np.floor(bins * (np.exp(m[:, j]) - lo[j]) / wid[j])
        b = np.clip(np.nan_to_num(b, nan=0.0, posinf=bins - 1, neginf=0.0), 0, bins - 1).astype(np.int64)
        b = np.where(key % 2 == 1, bins - 1 - b, b)
        key = key * bins + b
    return key


def valid_voxels(y, weights=None):
    y = np.asarray(y, dtype=np.float32)
    ok = np.all(np.isfinite(y), axis=1) & (np.max(y, axis=1) > 0)
    if weights is not None:
        w = np.asarray(weights, dtype=np.float32)
        ok &= np.all(np.isfinite(w) & (w >= 0), axis=1)
    return ok


def grouping(y, o, dims, bins, group_voxels, box_last, scale, weights=None):
    """(key [V], order [V] (voxel at each position), group [V] of each voxel,
    mu [G][D], sd [G][D] (fp32 values as float64), count [G])."""
    V = y.shape[0]
    m, s = summaries(o, dims)
    lo, wid = box32(box_last, HEAD_SLOTS[dims])
    key = cell_keys(m, bins, lo, wid)
    bad = ~valid_voxels(y, weights) | ~np.all(np.isfinite(m) & np.isfinite(s), axis=1)
    key = np.where(bad, bins ** dims, key)
    order = np.argsort(key, kind="stable")
    group = np.empty(V, dtype=np.int64)
    group[order] = np.arange(V) // group_voxels
    G = -(-V // group_voxels)
    mu = np.zeros((G, dims))
    sd = np.ones((G, dims))
    cnt = np.zeros(G, dtype=np.int64)
    for g in range(G):
        mem = order[g * group_voxels:(g + 1) * group_voxels]
        mem = mem[~bad[mem]]
        cnt[g] = mem.size
        if mem.size:
            mu_g = m[mem].sum(axis=0) / mem.size
            var = np.maximum(s[mem].sum(axis=0) / mem.size - mu_g * mu_g, 1e-12)
            mu[g] = mu_g.astype(np.float32)
            sd[g] = (np.sqrt(var) * scale).astype(np.float32)
    return key, order, group, mu, sd, cnt


def bank_rows(g, mu_g, sd_g, cnt_g, models, boxes, dims, n_draws, share, seed):
    """Rows of group g: theta [M n][8] (fp32, slot order, NaN unused), log w
    [M n], valid [M n]."""
    M = len(models)
    theta = np.full((M * n_draws, ora.NSLOT), np.nan, dtype=np.float32)
    logw = np.zeros(M * n_draws)
    valid = np.ones(M * n_draws, dtype=bool)
    i = np.arange(n_draws, dtype=np.uint32)
    for mi, model in enumerate(models):
        slots = MODEL_SLOTS[model]
        np_ = len(slots)
        lo, wid = box32(boxes[mi], slots)
        # head parameter of each model parameter (k4 without one under a four-parameter head)
        dim_of = [0, 1, 2, dims - 1] if np_ == 4 else [0, 1, 2, 3 if dims == 5 else -1, dims - 1]
        ctr = np.stack([i, np.full(n_draws, g, np.uint32), np.full(n_draws, 3, np.uint32),
                        np.full(n_draws, mi << 16, np.uint32)], axis=1)
        w = ora.philox(ctr, seed).astype(np.uint64)
        if np_ > 4:
            ctr[:, 3] |= 1
            v = ora.philox(ctr, seed).astype(np.uint64)
        else:
            v = np.zeros_like(w)
        u0 = ((w[:, 0] & 255) | (w[:, 1] & 255) << 8 | (w[:, 2] & 255) << 16).astype(np.float64) * 2.0 ** -24
        u = np.concatenate([(w >> 8), (v[:, :3] >> 8)], axis=1).astype(np.float64) * 2.0 ** -24  # u_0..u_6
        prior = (u0 < share) | (cnt_g == 0)
        th = np.zeros((n_draws, np_), dtype=np.float32)
        z = np.zeros((n_draws, np_))
        ok = np.ones(n_draws, dtype=bool)
        L = np.zeros(n_draws)
        for p_ in range(np_):
            d = dim_of[p_]
            uni = prior | (d < 0) | (wid[p_] == 0.0)
            up = np.where(prior | (wid[p_] == 0.0), u[:, p_], u[:, 6])
            th_u = (lo[p_] + up * wid[p_]).astype(np.float32)
            q = p_ // 2
            r = np.sqrt(-2.0 * np.log(u[:, 2 * q] + 2.0 ** -24))
            ang = 2.0 * math.pi * u[:, 2 * q + 1]
            nrm = r * (np.sin(ang) if p_ % 2 else np.cos(ang))
            zg = (mu_g[d] + sd_g[d] * nrm) if d >= 0 else np.zeros(n_draws)
            th_g = np.exp(zg).astype(np.float32)
            th[:, p_] = np.where(uni, th_u, th_g)
            with np.errstate(divide="ignore"):
                z[:, p_] = np.where(uni, np.log(th[:, p_].astype(np.float64)), zg)
            ok &= uni | ((th_g >= np.float32(lo[p_])) & (th_g.astype(np.float64) <= lo[p_] + wid[p_]))
            if d >= 0 and wid[p_] > 0.0 and cnt_g > 0:
                with np.errstate(invalid="ignore"):
                    t = (z[:, p_] - mu_g[d]) / sd_g[d]
                    L = L + (-0.5 * t * t - math.log(sd_g[d]) - 0.5 * math.log(2.0 * math.pi) - z[:, p_]
                             + math.log(wid[p_]))
        if cnt_g > 0:
            with np.errstate(divide="ignore", invalid="ignore"):
                if share == 0.0:
                    lw = -L
                else:
                    lw = -np.logaddexp(np.log(share), np.log1p(-share) + L)
            lw = np.where(np.isfinite(L), lw, np.where(L > 0, -np.inf, -math.log(share) if share > 0 else np.inf))
        else:
            lw = np.zeros(n_draws)
        lw = np.where(ok, lw, -np.inf)
        rows = slice(mi * n_draws, (mi + 1) * n_draws)
        theta[rows][:, list(slots)] = th
        logw[rows] = lw
        valid[rows] = ok
    return theta, logw, valid


def bank_curves(theta, valid, models, n_draws, input_fn, dt, frame_times):
    """FP64 frame averages [M n][F] of the valid rows (NaN for invalid ones)."""
    F = np.asarray(frame_times).size - 1
    x = np.full((theta.shape[0], F), np.nan)
    for mi, model in enumerate(models):
        rows = np.arange(mi * n_draws, (mi + 1) * n_draws)
        rows = rows[valid[rows]]
        if rows.size:
            x[rows] = ora.simulate(model, theta[rows], input_fn, dt, frame_times)
    return x


def infer_bank_learned(y, frame_times, input_fn, dt, models, boxes, o, n_draws, accept_frac, seed, *, dims=4,
                       bins=4, group_voxels=256, prior_share=0.1, sd_scale=1.0, lam=ora.DEFAULT_LAMBDA,
                       floor=ora.DEFAULT_FLOOR, l1=False, weights=None, accept_below=None, voxels=None,
                       first_group=0):
    """The whole method for the voxels listed in `voxels` (default: all; the
    grouping always uses every voxel).  Returns a dict: group [V], key [V],
    mu, sd, count [G], and per listed voxel accept_idx (rows of its group's
    bank), accept_dist (FP64), threshold, moments [M][8][2], model_prob [M],
    ess and the distances to every row of its group's bank; plus bank(g) ->
    (theta, logw, x) for checking."""
    y = np.asarray(y, dtype=np.float32)
    V, F = y.shape
    M = len(models)
    boxes = np.asarray(boxes, dtype=np.float64).reshape(M, ora.NSLOT, 2)
    key, order, group, mu, sd, cnt = grouping(y, o, dims, bins, group_voxels, boxes[-1], sd_scale, weights)
    n = ora.accept_count(M * n_draws, accept_frac)
    cp = np.asarray(input_fn, dtype=np.float32)
    banks = {}

    def bank(g):
        if g not in banks:
            th, lw, ok = bank_rows(first_group + g, mu[g], sd[g], cnt[g], models, boxes, dims, n_draws, prior_share,
                                   seed)
            banks[g] = (th, lw, bank_curves(th, ok, models, n_draws, cp, dt, frame_times))
        return banks[g]

    vox = np.arange(V) if voxels is None else np.asarray(voxels)
    out = {"group": group, "key": key, "mu": mu, "sd": sd, "count": cnt, "n": n, "bank": bank,
           "accept_idx": np.full((vox.size, n), -1, dtype=np.int64), "accept_dist": np.full((vox.size, n), np.nan),
           "threshold": np.full(vox.size, np.nan), "moments": np.full((vox.size, M, ora.NSLOT, 2), np.nan),
           "model_prob": np.full((vox.size, M), np.nan), "ess": np.full(vox.size, np.nan),
           "distances": [None] * vox.size}
    ok_vox = valid_voxels(y, weights)
    for k, v in enumerate(vox):
        if not ok_vox[v]:
            continue
        th, lw, x = bank(int(group[v]))
        if weights is None:
            wv = ora.weights(y[v], frame_times, dt, cp.size, lam=lam, floor=floor)
        else:
            wv = np.asarray(weights[v], dtype=np.float32).astype(np.float64)
        r = y[v].astype(np.float64) - x
        with np.errstate(invalid="ignore"):
            d = (np.sqrt(wv) * np.abs(r)).sum(axis=1) if l1 else (wv * r * r).sum(axis=1)
        d32 = np.where(np.isnan(d), np.inf, d).astype(np.float32)
        out["distances"][k] = d
        sel = np.lexsort((np.arange(d.size), d32))[:n]
        out["accept_idx"][k] = sel
        out["accept_dist"][k] = d[sel]
        out["threshold"][k] = d32[sel[-1]]
        out["moments"][k], out["model_prob"][k], out["ess"][k] = summarize_rows(
            sel, d32, th, lw, models, n_draws, None if accept_below is None else accept_below[v])
    return out


def summarize_rows(sel, d32, theta, logw, models, n_draws, below=None):
    """Weighted summaries of the accepted rows `sel` of one group's bank (see
    step 7): moments [M][8][2], model probabilities [M], ESS."""
    M = len(models)
    keep = np.asarray(sel)
    if below is not None:
        keep = keep[d32[keep] <= np.float32(below)]
    keep = keep[np.isfinite(logw[keep])]
    mom = np.full((M, ora.NSLOT, 2), np.nan)
    prob = np.full(M, np.nan)
    if keep.size == 0:
        return mom, prob, np.nan
    lw = logw[keep]
    w = np.exp(lw - lw.max())
    sw = w.sum()
    for mi, model in enumerate(models):
        mk = (keep // n_draws) == mi
        prob[mi] = w[mk].sum() / sw
        if not mk.any():
            continue
        t = theta[keep[mk]].astype(np.float64)
        t[:, 5] = t[:, 0] * t[:, 2] / (t[:, 1] + t[:, 2])
        used = list(MODEL_SLOTS[model]) + [5]
        ww = w[mk]
        mean = (ww[:, None] * t[:, used]).sum(axis=0) / ww.sum()
        var = (ww[:, None] * (t[:, used] - mean) ** 2).sum(axis=0) / ww.sum()
        mom[mi, used, 0] = mean
        mom[mi, used, 1] = var
    return mom, prob, sw * sw / (w * w).sum()
