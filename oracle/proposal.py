"""FP64 oracle of the learned proposal and importance-weighted ABC.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain numpy, FP64,
written from the definitions below; it shares no code with the GPU library.

This part is not in the paper.  It is an amortised importance sampler for the
prior draws of Alg. 1 (lines 1-2): a multilayer perceptron maps a voxel's
observed TAC to a mixture of Gaussians over the log of the free parameters,
draws come from that mixture instead of the prior, and each accepted draw is
weighted by prior / proposal (the usual importance weight, so the ABC target
is unchanged).  Definitions:

* features: x_f = log1p(max(y_f, 0)), zero-padded to NF = 32 inputs;
* network: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), o = h2 W3 + b3, widths
  32 -> 256 -> 256 -> 72 (8 mixture logits, 8 x 4 means, 8 x 4 raw scales);
* mixture over z = log(theta) of the D = 4 free parameters (K1, k2, k3, vB of
  the irreversible 2TCM): weights softmax(logits); log sd = LS0 + (LS1 - LS0)
  sigmoid(raw) (a smooth clamp to [LS0, LS1]).  A head over D = 5 parameters
  (K1, k2, k3, k4, vB of the reversible 2TCM) reads outputs 8 + 5 c + j
  (means) and 48 + 5 c + j (raw scales) instead (88 outputs in use);
* training loss: mean negative log density of z = log(theta) of the training
  draws (clamped at 1e-6 before the log), minimised with Adam;
* inference-time options: an sd scale s (every component's log sd + log s,
  a wider proposal) and a defensive prior share a in [0, 1]: the proposal is
  a p(theta) + (1 - a) q(theta), a mixture with the prior (Hesterberg's
  defensive importance sampling), which bounds every weight by 1 / a;
* draws (voxel v, draw i): one Philox4x32-10 block, counter (i, v, 2, 0),
  key = seed, words w0..w3; u0 = ((w0 & 255) | (w1 & 255) << 8 | (w2 & 255)
  << 16) 2^-24 from the low bytes, u_j = (w_j >> 8) 2^-24 from the high 24
  bits.  If u0 < a the draw is from the prior: theta_j = fp32(lo_j + u_j
  (hi_j - lo_j)) and z_j = log theta_j.  Otherwise the component is the first
  c with a + (1 - a) cumsum(pi)_c > u0; two Box-Muller pairs n_{2p}, n_{2p+1}
  = r cos / sin(2 pi u_{2p+1}), r = sqrt(-2 ln(u_{2p} + 2^-24)); z_j = mu_cj
  + sd_cj n_j; theta_j = fp32(exp(z_j)); a draw outside the prior box (fp32
  bounds) has weight 0;
* weight: with L = log q(z) - sum_j z_j + sum_j log(hi_j - lo_j) (the log
  ratio proposal / prior in theta space; sum_j z_j is the Jacobian of
  theta = exp(z)), log w = -log(a + (1 - a) e^L); L = -inf when some
  theta_j = 0.  Normalised over the accepted draws with a max shift in FP64;
* summaries: weighted mean sum w t / sum w, weighted variance
  sum w (t - mean)^2 / sum w, effective sample size (sum w)^2 / sum w^2.
"""
from __future__ import annotations

import math

import numpy as np

NF, H, NOUT, C, D = 32, 256, 72, 8, 4
LS0, LS1 = -6.0, 2.0
FREE_SLOTS = (0, 1, 2, 4)  # K1, k2, k3, vB of the irreversible 2TCM


def head_slots(dims: int = D):
    """theta slots of a head's parameters: (K1, k2, k3, vB) or (K1, k2, k3, k4, vB)."""
    return {4: (0, 1, 2, 4), 5: (0, 1, 2, 3, 4)}[dims]


def head_outputs(dims: int = D) -> int:
    """Outputs in use by a head over dims parameters."""
    return C + 2 * C * dims


def init_params(rng: np.random.Generator, dims: int = D) -> dict:
    """He-normal weights, zero biases (FP64)."""
    no = head_outputs(dims)
    return {"W1": rng.standard_normal((NF, H)) * math.sqrt(2.0 / NF), "b1": np.zeros(H),
            "W2": rng.standard_normal((H, H)) * math.sqrt(2.0 / H), "b2": np.zeros(H),
            "W3": rng.standard_normal((H, no)) * math.sqrt(1.0 / H), "b3": np.zeros(no)}


def features(y: np.ndarray) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros((y.shape[0], NF))
    x[:, :y.shape[1]] = np.log1p(np.maximum(y, 0.0))
    return x


def forward(p: dict, x: np.ndarray):
    a1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(a2, 0.0)
    o = h2 @ p["W3"] + p["b3"]
    return o, (x, a1, h1, a2, h2)


def mixture(o: np.ndarray, sd_scale: float = 1.0, dims: int = D):
    """(log pi [B][C], mu [B][C][dims], log sd [B][C][dims]) of network outputs."""
    logits = o[:, :C]
    m = logits.max(axis=1, keepdims=True)
    logpi = logits - m - np.log(np.exp(logits - m).sum(axis=1, keepdims=True))
    mu = o[:, C:C + C * dims].reshape(-1, C, dims)
    raw = o[:, C + C * dims:C + 2 * C * dims].reshape(-1, C, dims)
    logsd = LS0 + (LS1 - LS0) / (1.0 + np.exp(-raw))
    if sd_scale != 1.0:
        logsd = logsd + math.log(sd_scale)
    return logpi, mu, logsd


def log_density(o: np.ndarray, z: np.ndarray, sd_scale: float = 1.0) -> np.ndarray:
    """log q(z) per row (the mixture density of z; the head's size is z's width)."""
    logpi, mu, logsd = mixture(o, sd_scale, dims=z.shape[1])
    t = (z[:, None, :] - mu) * np.exp(-logsd)
    comp = logpi + (-0.5 * t * t - logsd - 0.5 * math.log(2.0 * math.pi)).sum(axis=2)
    mx = comp.max(axis=1, keepdims=True)
    return (mx + np.log(np.exp(comp - mx).sum(axis=1, keepdims=True)))[:, 0]


def targets(theta: np.ndarray, dims: int = D) -> np.ndarray:
    """z = log(theta) of the head's parameters (theta clamped at 1e-6)."""
    t = np.asarray(theta, dtype=np.float64)[:, list(head_slots(dims))]
    return np.log(np.maximum(t, 1e-6))


def loss_and_grad(p: dict, x: np.ndarray, z: np.ndarray):
    """Mean negative log density and its gradient with respect to every
    parameter (a head over z's width of parameters)."""
    B, Dz = x.shape[0], z.shape[1]
    o, (x, a1, h1, a2, h2) = forward(p, x)
    logpi, mu, logsd = mixture(o, dims=Dz)
    sd_inv = np.exp(-logsd)
    t = (z[:, None, :] - mu) * sd_inv
    comp = logpi + (-0.5 * t * t - logsd - 0.5 * math.log(2.0 * math.pi)).sum(axis=2)
    mx = comp.max(axis=1, keepdims=True)
    lse = mx + np.log(np.exp(comp - mx).sum(axis=1, keepdims=True))
    loss = -lse.mean()
    r = np.exp(comp - lse)                     # responsibilities [B][C]
    do = np.zeros_like(o)
    do[:, :C] = (np.exp(logpi) - r) / B        # d(-log q)/d logits
    do[:, C:C + C * Dz] = (-(r[:, :, None] * t * sd_inv) / B).reshape(B, -1)
    s = (logsd - LS0) / (LS1 - LS0)            # sigmoid(raw)
    dlogsd = r[:, :, None] * (1.0 - t * t) / B
    do[:, C + C * Dz:C + 2 * C * Dz] = (dlogsd * (LS1 - LS0) * s * (1.0 - s)).reshape(B, -1)
    g = {"W3": h2.T @ do, "b3": do.sum(axis=0)}
    dh2 = (do @ p["W3"].T) * (a2 > 0.0)
    g["W2"], g["b2"] = h1.T @ dh2, dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"].T) * (a1 > 0.0)
    g["W1"], g["b1"] = x.T @ dh1, dh1.sum(axis=0)
    return loss, g


def adam(p: dict, g: dict, state: dict, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) in place; state holds m, v and t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1.0 - b1) * g[k]
        v[...] = b2 * v + (1.0 - b2) * g[k] * g[k]
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)


def draws(o_v: np.ndarray, words: np.ndarray, lo=None, hi=None, prior_share: float = 0.0, sd_scale: float = 1.0):
    """Proposal draws of one voxel: z [n][D] (FP64), theta [n][D] (fp32) from the
    voxel's network output o_v [72], Philox words [n][4] and, for the
    defensive share, the fp32 prior box lo, hi [D]."""
    logpi, mu, logsd = mixture(o_v[None, :], sd_scale)
    a = float(prior_share)
    cum = a + (1.0 - a) * np.cumsum(np.exp(logpi[0]))
    w = words.astype(np.uint64)
    u0 = ((w[:, 0] & 255) | (w[:, 1] & 255) << 8 | (w[:, 2] & 255) << 16).astype(np.float64) * 2.0 ** -24
    u = (w >> 8).astype(np.float64) * 2.0 ** -24
    c = np.minimum(np.searchsorted(cum, u0, side="right"), C - 1)
    nrm = np.empty((words.shape[0], D))
    for q in range(2):
        r = np.sqrt(-2.0 * np.log(u[:, 2 * q] + 2.0 ** -24))
        nrm[:, 2 * q] = r * np.cos(2.0 * math.pi * u[:, 2 * q + 1])
        nrm[:, 2 * q + 1] = r * np.sin(2.0 * math.pi * u[:, 2 * q + 1])
    z = mu[0][c] + np.exp(logsd[0][c]) * nrm
    th = np.exp(z).astype(np.float32)
    from_prior = u0 < a
    if from_prior.any():
        lo64, hi64 = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
        th[from_prior] = (lo64 + u[from_prior] * (hi64 - lo64)).astype(np.float32)
        with np.errstate(divide="ignore"):
            z[from_prior] = np.log(th[from_prior].astype(np.float64))
    return z, th


def log_weight(o_v: np.ndarray, z: np.ndarray, lo=None, hi=None, prior_share: float = 0.0,
               sd_scale: float = 1.0) -> np.ndarray:
    """log w = -log(a + (1 - a) q(theta) / p(theta)) of draws z [n][D]."""
    a = float(prior_share)
    logvol = 0.0 if lo is None else float(np.sum(np.log(np.asarray(hi, np.float64) - np.asarray(lo, np.float64))))
    L = np.full(z.shape[0], -np.inf)
    fin = np.all(np.isfinite(z), axis=1)
    if fin.any():
        L[fin] = (log_density(np.repeat(o_v[None, :], int(fin.sum()), axis=0), z[fin], sd_scale)
                  - z[fin].sum(axis=1) + logvol)
    if a == 0.0:
        return -L
    with np.errstate(divide="ignore"):
        return -np.logaddexp(math.log(a), np.log1p(-a) + L)


def weighted_summary(theta: np.ndarray, logw: np.ndarray):
    """Weighted mean, variance (both per column) and ESS, FP64 with a max shift."""
    w = np.exp(logw - logw.max())
    sw = w.sum()
    mean = (w[:, None] * theta).sum(axis=0) / sw
    var = (w[:, None] * (theta - mean) ** 2).sum(axis=0) / sw
    return mean, var, sw * sw / (w * w).sum()


def philox_words(v: int, n: int, seed: int) -> np.ndarray:
    """Words [n][4] of the proposal draws i = 0..n-1 of voxel v (stream 2)."""
    import oracle as ora
    i = np.arange(n, dtype=np.uint32)
    ctr = np.stack([i, np.full(n, v, np.uint32), np.full(n, 2, np.uint32), np.zeros(n, np.uint32)], axis=1)
    return ora.philox(ctr, seed)


def infer_is(y_v, frame_times, input_fn, dt, box, o_v, n_draws, accept_frac, seed, v_global, lam=None,
             prior_share=0.0, sd_scale=1.0, l1=False, weights_v=None, accept_below=None):
    """Importance-weighted fixed-budget ABC of one voxel (irreversible 2TCM):
    n_draws proposal draws, the n closest valid ones accepted (ties to the lower
    draw index), weighted summaries.  Distances as in the plain method: the
    noise-weighted L2 sum_f w_f (y_f - x_f)^2, or L1 sum_f sqrt(w_f) |y_f - x_f|,
    with the default weights or the caller's weights_v.  With accept_below = h,
    only the accepted draws whose distance (rounded to fp32, as the ranking
    keys are) is at most h enter the summaries: ABC at a given threshold, the
    indicator form of Eq. (7).  Returns (accepted indices, moments [8][2] with
    Ki in slot 5 and NaN in unused slots, ESS, distances of every draw)."""
    import oracle as ora
    lam = ora.DEFAULT_LAMBDA if lam is None else lam
    lo = np.array([np.float32(box[s][0]) for s in FREE_SLOTS], dtype=np.float64)
    hi = np.array([np.float32(box[s][1]) for s in FREE_SLOTS], dtype=np.float64)
    o_v = np.asarray(o_v, dtype=np.float64)
    words = philox_words(v_global, n_draws, seed)
    z, th4 = draws(o_v, words, lo, hi, prior_share, sd_scale)
    valid = np.all((th4 >= lo.astype(np.float32)) & (th4 <= hi.astype(np.float32)), axis=1)
    theta = np.full((n_draws, 8), np.nan, dtype=np.float32)
    theta[:, FREE_SLOTS] = th4
    cp = np.asarray(input_fn, dtype=np.float32)
    y = np.asarray(y_v, dtype=np.float32)
    if weights_v is None:
        w = ora.weights(y, frame_times, dt, cp.size, lam=lam)
    else:
        w = np.asarray(weights_v, dtype=np.float32).astype(np.float64)
    d = np.full(n_draws, np.inf)
    if valid.any():
        x = ora.simulate(ora.M_2TCM_IRR, theta[valid], cp, dt, frame_times)
        r = y.astype(np.float64) - x
        d[valid] = (np.sqrt(w) * np.abs(r)).sum(axis=1) if l1 else (w * r * r).sum(axis=1)
    n = ora.accept_count(n_draws, accept_frac)
    order = np.lexsort((np.arange(n_draws), d))[:n]
    keep = order[np.isfinite(d[order])]
    if accept_below is not None:
        keep = keep[d[keep].astype(np.float32) <= np.float32(accept_below)]
    t = theta[keep].astype(np.float64)
    t[:, 5] = t[:, 0] * t[:, 2] / (t[:, 1] + t[:, 2])
    mom = np.full((8, 2), np.nan)
    ess = np.nan
    if keep.size:
        cols = [0, 1, 2, 4, 5]
        mean, var, ess = weighted_summary(t[:, cols], log_weight(o_v, z[keep], lo, hi, prior_share, sd_scale))
        mom[cols, 0] = mean
        mom[cols, 1] = var
    return order, mom, ess, d
