"""GPU parity of the shared bank drawn from a learned proposal
(vpet_abc_infer_bank_learned) against oracle/learned_bank.py, through the C
ABI.

Tolerances.  The grouping (cells, order, group Gaussians rounded to fp32) and
the bank draws are the same arithmetic on both sides up to the last bits of
FP64 library functions, so groups are identical and a bank row's fp32
parameters are identical unless an FP64 value lands within an ulp of an fp32
rounding boundary (at most a 1e-4 fraction of rows, and then by one fp32 ulp);
log weights agree within 1e-9.  Selections follow the swap rule of the plain
method: the accepted sets are identical except for rows within 1e-5 (relative)
of the oracle's threshold, and the summaries are compared with the oracle's
reduction of the GPU's own set (weighted means, variances and ESS within
1e-5 relative, probabilities within 1e-6).
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import THRESH_RTOL, spread_sample

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2603_14859_amd as V  # noqa: E402
import oracle as ora  # noqa: E402
import oracle.learned_bank as lb  # noqa: E402
import oracle.proposal as prop  # noqa: E402

DEV = torch.device("cuda:0")
IRR, REV = W.M_2TCM_IRR, W.M_2TCM_REV


def _volume(n, seed, models=(IRR,), sched=W.SCHED_30x50):
    ft = W.frame_times(sched)
    dt = 0.2
    _, cp = W.grid(dt, float(np.sum(sched)))
    rng = np.random.default_rng(seed)
    rev = rng.random(n) < 0.5 if len(models) > 1 else np.zeros(n, bool)
    th = W.true_params(rng, n, REV, W.box_array([REV])[0])
    th[~rev, 3] = 0.0
    clean = np.empty((n, ft.size - 1))
    for m, sel in ((IRR, ~rev), (REV, rev)):
        if sel.any():
            clean[sel] = ora.simulate(m, th[sel], cp, dt, ft)
    y = W.add_noise(clean, ft, rng.standard_normal(clean.shape))
    return ft, cp, dt, th, y, rng


def _outputs(th, rng, dims, spread=0.3, sd=0.3):
    n = th.shape[0]
    o = np.zeros((n, 96), dtype=np.float32)
    o[:, :prop.C] = rng.standard_normal((n, prop.C))
    z0 = np.log(np.maximum(th[:, list(prop.head_slots(dims))], 1e-3))
    o[:, prop.C:prop.C + prop.C * dims] = (np.repeat(z0[:, None, :], prop.C, axis=1)
                                           + spread * rng.standard_normal((n, prop.C, dims))).reshape(n, -1)
    s = (math.log(sd) - prop.LS0) / (prop.LS1 - prop.LS0)
    o[:, prop.C + prop.C * dims:prop.C + 2 * prop.C * dims] = (math.log(s / (1 - s))
                                                               + 0.3 * rng.standard_normal((n, prop.C * dims)))
    return o


def _run(y, ft, cp, dt, models, o, n_draws, p, seed, *, sample=None, weights=None, below=None, distance="l2",
         scan="auto", **gk):
    boxes = W.box_array(list(models))
    res = V.infer_bank_learned(torch.from_numpy(y).to(DEV), ft, cp, dt, list(models), boxes,
                               torch.from_numpy(o).to(DEV), n_draws, p, seed, debug=True, return_bank=True,
                               weights=None if weights is None else torch.from_numpy(weights).to(DEV),
                               accept_below=None if below is None else torch.from_numpy(below).to(DEV),
                               distance=distance, bank_scan=scan, **gk)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()}
    rows = np.arange(y.shape[0]) if sample is None else np.asarray(sample)
    ref = lb.infer_bank_learned(y, ft, cp, dt, list(models), boxes, o.astype(np.float64), n_draws, p, seed,
                                weights=weights, accept_below=below, voxels=rows, l1=distance == "l1", **gk)
    return g, ref, rows


def _check(g, ref, rows, models, n_draws, below=None, check_bank=True):
    """Every listed voxel against the oracle under the swap rule; the bank
    rows of their groups draw by draw."""
    assert np.array_equal(g["group"], ref["group"]), "group assignment"
    n_theta_diff = n_rows = 0
    if check_bank:
        for gi in sorted(set(int(ref["group"][v]) for v in rows)):
            th_o, lw_o, _ = ref["bank"](gi)
            th_g, lw_g = g["bank_theta"][gi], g["bank_logw"][gi]
            same = (th_g.view(np.uint32) == th_o.view(np.uint32)) | (np.isnan(th_g) & np.isnan(th_o))
            diff = ~same.all(axis=1)
            n_theta_diff += int(diff.sum())
            n_rows += th_o.shape[0]
            if diff.any():  # one fp32 ulp at most
                a, b = th_g[diff].astype(np.float64), th_o[diff].astype(np.float64)
                ulp = np.spacing(np.abs(b).astype(np.float32)).astype(np.float64)
                assert np.all((np.abs(a - b) <= ulp) | (np.isnan(a) & np.isnan(b))), f"group {gi}: bank draws"
            fin = np.isfinite(lw_o)
            assert np.array_equal(fin, np.isfinite(lw_g)), f"group {gi}: invalid rows"
            assert np.allclose(lw_g[fin], lw_o[fin], rtol=1e-9, atol=1e-9), f"group {gi}: log weights"
        assert n_theta_diff <= max(2, 1e-4 * n_rows), (n_theta_diff, n_rows)
    swaps = 0
    for k, v in enumerate(rows):
        gm, gp, ge = g["moments"][v].astype(np.float64), g["model_prob"][v].astype(np.float64), float(g["ess"][v])
        if np.isnan(ref["threshold"][k]):  # invalid voxel
            assert np.isnan(gm).all() and np.isnan(gp).all() and np.isnan(ge) and (g["accept_idx"][v] == -1).all()
            continue
        a_g, a_o = set(g["accept_idx"][v].tolist()), set(ref["accept_idx"][k].tolist())
        mom, prob, ess = ref["moments"][k], ref["model_prob"][k], ref["ess"][k]
        if a_g != a_o:
            # only rows within 1e-5 (relative) of the oracle's threshold may
            # swap; the summaries are then the oracle's reduction of the
            # GPU's own set
            swaps += 1
            d = ref["distances"][k]
            h = ref["threshold"][k]
            for q in a_g ^ a_o:
                assert abs(d[q] - h) <= THRESH_RTOL * h, f"voxel {v}: row {q} swapped far from the threshold"
            th_o, lw_o, _ = ref["bank"](int(ref["group"][v]))
            d32 = np.where(np.isnan(d), np.inf, d).astype(np.float32)
            mom, prob, ess = lb.summarize_rows(np.array(sorted(a_g)), d32, th_o, lw_o, list(models), n_draws,
                                               None if below is None else below[v])
        assert np.array_equal(np.isnan(gm), np.isnan(mom)), f"voxel {v}: NaN pattern"
        ok = ~np.isnan(mom)
        assert np.allclose(gm[ok], mom[ok], rtol=1e-5, atol=1e-7), f"voxel {v}: moments"
        assert np.allclose(gp, prob, rtol=0, atol=1e-6, equal_nan=True), f"voxel {v}: model probabilities"
        if np.isnan(ess):
            assert np.isnan(ge)
        else:
            assert ge == pytest.approx(ess, rel=1e-5)
    return swaps, n_theta_diff


@pytest.mark.parametrize("dims,bins,models", [(4, 3, (IRR,)), (4, 2, (IRR, REV)), (5, 2, (IRR, REV)),
                                              (5, 1, (REV,))])
def test_learned_bank_parity(dims, bins, models):
    """700 voxels (two whole groups of 256 and a ragged third), an invalid
    voxel and one without a positive frame; both models and both heads."""
    ft, cp, dt, th, y, rng = _volume(700, 40 + dims + bins, models)
    o = _outputs(th, rng, dims)
    y[5, 3] = np.nan
    y[6] = -1.0
    g, ref, rows = _run(y, ft, cp, dt, models, o, 3000, 0.01, 77, dims=dims, bins=bins, group_voxels=256,
                        prior_share=0.15, sd_scale=1.3)
    swaps, nd = _check(g, ref, rows, models, 3000)
    print(f"[learned bank] dims={dims} bins={bins} models={models}: threshold swaps {swaps}, "
          f"bank rows off by one ulp {nd}, fallback voxels {g['fallback_voxels']}")
    assert g["group"][5] == g["group"][6] == 2  # invalid voxels sort last


@pytest.mark.parametrize("sched", [W.SCHED_22x60, W.SCHED_40x90])
def test_learned_bank_parity_other_frame_counts(sched):
    """22 and 40 frames (bank rows padded to 24 and 40 values, so that a
    row's values and operands do not fill whole 64-lane store runs) and a
    ragged last wavefront of bank rows (700 per model)."""
    ft, cp, dt, th, y, rng = _volume(300, 61 + len(sched), (IRR, REV), sched=sched)
    o = _outputs(th, rng, 5)
    g, ref, rows = _run(y, ft, cp, dt, (IRR, REV), o, 700, 0.02, 31, dims=5, bins=1, group_voxels=256,
                        prior_share=0.2, sd_scale=1.3)
    swaps, nd = _check(g, ref, rows, (IRR, REV), 700)
    print(f"[learned bank] {len(sched)} frames: threshold swaps {swaps}, bank rows off by one ulp {nd}, "
          f"fallback voxels {g['fallback_voxels']}")


def test_learned_bank_scans_agree_and_l1_weights_threshold():
    """The FP64 scan and the BF16 contraction scan give the same outputs bit
    for bit; the L1 distance with caller weights and ABC at given thresholds
    against the oracle."""
    ft, cp, dt, th, y, rng = _volume(600, 51, (IRR, REV))
    o = _outputs(th, rng, 5, spread=0.2, sd=0.4)
    gk = dict(dims=5, bins=2, group_voxels=256, prior_share=0.2, sd_scale=1.2)
    outs = []
    for scan in ("f64", "bf16"):
        res = V.infer_bank_learned(torch.from_numpy(y).to(DEV), ft, cp, dt, [IRR, REV], W.box_array([IRR, REV]),
                                   torch.from_numpy(o).to(DEV), 2500, 0.01, 5, debug=True, bank_scan=scan, **gk)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in res.items() if torch.is_tensor(v)})
    for k in ("accept_idx", "accept_dist", "threshold", "moments", "model_prob", "ess"):
        assert np.array_equal(outs[0][k], outs[1][k], equal_nan=True), k
    w = rng.uniform(0.3, 2.0, y.shape).astype(np.float32)
    w[7, 2] = -1.0  # invalid voxel
    sample = np.arange(0, 600, 37)
    g, ref, rows = _run(y, ft, cp, dt, (IRR, REV), o, 2500, 0.01, 5, sample=sample, weights=w, distance="l1", **gk)
    _check(g, ref, rows, (IRR, REV), 2500)
    # given thresholds: midway between two of the oracle's accepted distances
    ref0 = lb.infer_bank_learned(y, ft, cp, dt, [IRR, REV], W.box_array([IRR, REV]), o.astype(np.float64), 2500,
                                 0.01, 5, voxels=sample, **gk)
    below = np.full(600, np.inf, dtype=np.float32)
    for k, v in enumerate(sample):
        d = np.sort(ref0["accept_dist"][k])
        j = 1 + (3 * k) % 40
        below[v] = np.float32(0.5 * (d[j - 1] + d[j]))
    below[sample[1]] = 0.0
    g, ref, rows = _run(y, ft, cp, dt, (IRR, REV), o, 2500, 0.01, 5, sample=sample, below=below, **gk)
    _check(g, ref, rows, (IRR, REV), 2500, below=below)
    assert np.isnan(g["moments"][sample[1]]).all() and np.isnan(g["ess"][sample[1]])


def test_learned_bank_full_size_sampled():
    """1,048,576 voxels x 20,000-row banks (one per group of 1024 voxels,
    1024 groups, eight cells per parameter), 30 frames, 100 accepted; 32
    voxels spread over the volume against the oracle, none exempt."""
    cfg = W.CFG_LARGE
    ft, cp = cfg.frame_times, cfg.input_fn()
    from parity import large_volume
    th, y = large_volume(cfg)
    o = _outputs(th, np.random.default_rng(8), 4, spread=0.15, sd=0.25)
    sample = spread_sample(cfg.n_voxels, k=32, seed=8)
    g, ref, rows = _run(y, ft, cp, cfg.dt, (IRR,), o, 20_000, 0.005, cfg.infer_seed, sample=sample, dims=4, bins=8,
                        group_voxels=1024, prior_share=0.1, sd_scale=1.5)
    swaps, nd = _check(g, ref, rows, (IRR,), 20_000)
    print(f"[learned bank full size] swaps {swaps}, bank rows off by one ulp {nd}, "
          f"fallback voxels {g['fallback_voxels']}, median ESS {np.nanmedian(g['ess']):.1f}")
    assert np.isfinite(g["moments"][:, 0, 5, 0]).mean() > 0.999
