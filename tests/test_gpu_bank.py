"""GPU parity of the shared-bank form (Alg. 1 as printed: one bank of draws and
curves for every voxel) against the oracle's bank form, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from parity import MEAN_RTOL, THRESH_RTOL, bank_distances, check_voxels, large_volume, spread_sample  # noqa: F401

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2603_14859_amd as V  # noqa: E402

DEV = torch.device("cuda:0")
H = 0.2


def _inputs(sched, n_vox, model=W.M_2TCM_IRR, seed=5):
    import oracle as ora
    ft = W.frame_times(sched)
    _, cp = W.grid(H, float(np.sum(sched)))
    rng = np.random.default_rng(seed)
    th = W.true_params(rng, n_vox, model, W.box_array([model])[0])
    clean = ora.simulate(model, th, cp, H, ft)
    return ft, cp, W.add_noise(clean, ft, rng.standard_normal(clean.shape))


def _bank_moments(models, th_bank, idx, n_draws):
    """FP64 summaries of an explicit accepted set drawn from the bank."""
    M = len(models)
    t = th_bank[np.asarray(idx)].astype(np.float64)
    t[:, 5] = t[:, 0] * t[:, 2] / (t[:, 1] + t[:, 2])
    m = np.asarray(idx) // n_draws
    mom = np.full((M, 8, 2), np.nan)
    prob = np.zeros(M)
    for mm in range(M):
        sel = t[m == mm]
        prob[mm] = sel.shape[0] / len(idx)
        if sel.shape[0]:
            mom[mm, :, 0] = sel.mean(axis=0)
            mom[mm, :, 1] = sel.var(axis=0, ddof=1) if sel.shape[0] > 1 else 0.0
            if models[mm] == W.M_1TCM:
                mom[mm, [2, 3, 5]] = np.nan
            elif models[mm] == W.M_2TCM_IRR:
                mom[mm, 3] = np.nan
            mom[mm, 6:] = np.nan
    return mom, prob


def _check(y, ft, cp, models, n_draws, p, seed, l1=False, weights=None, bank_pilot=0, scan="auto"):
    import oracle as ora
    boxes = W.box_array(list(models))
    th_g, x_g = V.bank_build(models, boxes, n_draws, seed, cp, ft, H)
    res = V.infer_bank(torch.from_numpy(y).to(DEV), ft, H, cp.size, models, n_draws, p, th_g, x_g,
                       distance="l1" if l1 else "l2", debug=True, bank_pilot=bank_pilot, bank_scan=scan,
                       weights=None if weights is None else torch.from_numpy(weights).to(DEV))
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()}
    o = ora.infer_bank(y, ft, cp, H, list(models), boxes, n_draws, p, seed, l1=l1, weights=weights)
    th_o, x_o = ora.bank(list(models), boxes, n_draws, seed, cp, H, ft)
    assert g["n"] == o["n"]
    swaps = 0
    for v in range(y.shape[0]):
        a_g, a_o = set(g["accept_idx"][v].tolist()), set(o["accept_idx"][v].tolist())
        if a_g != a_o:
            w = (ora.weights(y[v], ft, H, cp.size) if weights is None else weights[v].astype(np.float64))
            r = y[v].astype(np.float64) - x_o
            d = (np.sqrt(w) * np.abs(r)).sum(1) if l1 else (w * r * r).sum(1)
            h = o["threshold"][v]
            for gg in a_g ^ a_o:
                assert abs(d[gg] - h) <= THRESH_RTOL * h, f"voxel {v}: draw {gg} swapped far from the threshold"
            swaps += 1
            ref_mom, ref_prob = _bank_moments(list(models), th_o, g["accept_idx"][v], n_draws)
        else:
            ref_mom, ref_prob = o["moments"][v], o["model_prob"][v]
        gm = g["moments"][v].astype(np.float64)
        assert np.array_equal(np.isnan(gm), np.isnan(ref_mom)), f"voxel {v}: NaN pattern"
        ok = ~np.isnan(ref_mom)
        assert np.allclose(gm[ok], ref_mom[ok], rtol=1e-5, atol=1e-7), f"voxel {v}: moments"
        assert np.allclose(g["model_prob"][v], ref_prob, atol=1e-7, equal_nan=True)
    print(f"[bank parity] scan={scan} V={y.shape[0]} n={o['n']} voxels with threshold swaps: {swaps}, "
          f"exact fallbacks: {g['fallback_voxels']}")
    return g, o


def test_bank_build_matches_oracle():
    import oracle as ora
    models = [W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV]
    boxes = W.box_array(models)
    for sched in (W.SCHED_22x60, W.SCHED_30x50, [1.0, 2.0, 5.0]):
        ft = W.frame_times(sched)
        _, cp = W.grid(H, float(np.sum(sched)))
        th_g, x_g = V.bank_build(models, boxes, 3000, 77, cp, ft, H)
        th_o, x_o = ora.bank(models, boxes, 3000, 77, cp, H, ft)
        F = ft.size - 1
        xg = x_g.cpu().numpy()
        assert np.array_equal(th_g.cpu().numpy().view(np.uint32), th_o.view(np.uint32))
        err = np.abs(xg[:, :F] - x_o).max(axis=1) / np.abs(x_o).max(axis=1)
        assert err.max() < 1e-11, err.max()
        assert (xg[:, F:] == 0).all()


SCANS = ["f64", "bf16"]


@pytest.mark.parametrize("scan", SCANS)
def test_infer_bank_parity_30_frames(scan):
    # 300 voxels: two 256-voxel contraction blocks, the second ragged
    ft, cp, y = _inputs(W.SCHED_30x50, 300)
    _check(y, ft, cp, [W.M_2TCM_IRR], 20_000, 0.005, 14859, scan=scan)


@pytest.mark.parametrize("scan", SCANS)
@pytest.mark.parametrize("models", [(W.M_2TCM_IRR, W.M_2TCM_REV), (W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV)])
def test_infer_bank_parity_model_selection(models, scan):
    ft, cp, y = _inputs(W.SCHED_22x60, 120, model=W.M_2TCM_REV, seed=9)
    _check(y, ft, cp, list(models), 6000, 0.01, 3, scan=scan)


def test_infer_bank_scans_agree_on_odd_bank():
    """Bank size not a multiple of the 32-row tile; frame count 7 (padded to 8)."""
    ft, cp, y = _inputs([2.0, 3.0, 5.0, 5.0, 10.0, 10.0, 20.0], 333, seed=12)
    g1, _ = _check(y, ft, cp, [W.M_1TCM, W.M_2TCM_IRR], 4001, 0.01, 8, scan="f64")
    g2, _ = _check(y, ft, cp, [W.M_1TCM, W.M_2TCM_IRR], 4001, 0.01, 8, scan="bf16")
    same = sum(set(a.tolist()) == set(b.tolist()) for a, b in zip(g1["accept_idx"], g2["accept_idx"]))
    assert same >= y.shape[0] - 3


def test_infer_bank_l1_weights_and_short_schedule():
    ft, cp, y = _inputs([1.0, 2.0, 3.0, 6.0], 70, seed=2)
    _check(y, ft, cp, [W.M_2TCM_IRR], 5000, 0.01, 4, l1=True)
    w = np.random.default_rng(3).uniform(0.3, 2.0, y.shape).astype(np.float32)
    w[5, 1], w[8, 3], w[11, 0] = -0.5, np.nan, 0.0  # invalid, invalid, allowed
    g, _ = _check(y, ft, cp, [W.M_2TCM_IRR], 5000, 0.01, 4, weights=w)
    assert np.isnan(g["moments"][[5, 8]]).all() and np.isfinite(g["moments"][11, 0, 5, 0])


def test_infer_bank_forced_fallback_and_edges():
    ft, cp, y = _inputs(W.SCHED_22x60, 40, seed=7)
    y[5, 2] = np.nan
    y[6] = -1.0
    # a pilot over the whole bank leaves only about 16-25 rows below each
    # voxel's threshold, fewer than n = 60: (nearly) every voxel takes the
    # exact fallback path
    for scan in SCANS:
        g, _ = _check(y, ft, cp, [W.M_2TCM_IRR], 3000, 0.02, 11, bank_pilot=3000, scan=scan)
        for v in (5, 6):
            assert np.isnan(g["moments"][v]).all() and (g["accept_idx"][v] == -1).all()
        if scan == "f64":  # exactly 16 rows below each threshold: every valid voxel falls back
            assert g["fallback_voxels"] == y.shape[0] - 2
        else:
            assert g["fallback_voxels"] > (y.shape[0] - 2) // 2
        _check(y[:8], ft, cp, [W.M_2TCM_IRR, W.M_2TCM_REV], 150, 1.0, 5, scan=scan)  # p = 1: n = N = 300
        _check(y[:8], ft, cp, [W.M_2TCM_IRR], 7, 0.2, 5, scan=scan)                   # tiny bank, n = 1


def test_select_prunes_a_full_key_buffer():
    """About 580 near-copies of bank row 100 (its curve scaled by 1 + 1e-6 j)
    in the bank tiles that a 1024-row pilot does not sample, and a voxel equal
    to row 100: every near-copy lies below the voxel's pilot threshold, more
    than the re-ranking select's LDS key buffer holds (512 keys at n = 40), so
    the select prunes the buffer to its smallest keys mid-way instead of
    handing the voxel to the exact fallback.  The accepted set is row 100 and
    the 39 least-scaled copies."""
    ft, cp, y = _inputs(W.SCHED_30x50, 64, seed=21)
    models = [W.M_2TCM_IRR]
    th_g, x_g = V.bank_build(models, W.box_array(models), 8000, 5, cp, ft, H)
    # pilot tiles of 64 rows: floor(t 125 / 16) for t < 16 = 0, 7, 15, ...;
    # rows 64-447 and 512-703 lie in tiles 1-6 and 8-10
    rows = [r for r in list(range(64, 448)) + list(range(512, 704)) if r != 100]
    idx = torch.tensor(rows, device=DEV)
    scale = 1.0 + 1e-6 * torch.arange(1, len(rows) + 1, device=DEV, dtype=torch.float64)
    x_g[idx] = x_g[100].clone().unsqueeze(0) * scale.unsqueeze(1)
    th_g[idx] = th_g[100].clone()
    F = ft.size - 1
    y = y.copy()
    y[3] = x_g[100, :F].cpu().numpy().astype(np.float32)
    kw = dict(debug=True, bank_scan="bf16", bank_pilot=1024)
    res = V.infer_bank(torch.from_numpy(y).to(DEV), ft, H, cp.size, models, 8000, 0.005, th_g, x_g, **kw)
    one = V.infer_bank(torch.from_numpy(y[3:4]).to(DEV), ft, H, cp.size, models, 8000, 0.005, th_g, x_g, **kw)
    torch.cuda.synchronize()
    n = res["n"]
    assert n == 40
    want = {100} | set(rows[:n - 1])
    assert set(res["accept_idx"][3].cpu().numpy().tolist()) == want
    assert set(one["accept_idx"][0].cpu().numpy().tolist()) == want
    assert one["fallback_voxels"] == 0  # the select answered the voxel itself
    t0 = th_g[100].cpu().numpy().astype(np.float64)
    mom = one["moments"][0, 0].cpu().numpy().astype(np.float64)
    assert np.allclose(mom[:3, 0], t0[:3], rtol=1e-6) and np.allclose(mom[:3, 1], 0.0, atol=1e-12)
    print(f"[bank prune] exact fallbacks over the 64 voxels: {res['fallback_voxels']}, for the voxel alone: 0")


def test_infer_bank_limits():
    ft, cp, y = _inputs(W.SCHED_22x60, 2)
    th, x = V.bank_build([W.M_2TCM_IRR], W.box_array([W.M_2TCM_IRR]), 1000, 1, cp, ft, H)
    with pytest.raises(V.VpetError) as e:
        V.infer_bank(torch.from_numpy(y).to(DEV), ft, H, cp.size, [W.M_2TCM_IRR], 1000, 0.6, th, x)
    assert e.value.status == V.E_LIMIT
    with pytest.raises(V.VpetError) as e:
        V.infer_bank(torch.from_numpy(y).to(DEV), ft, H, cp.size, [W.M_2TCM_IRR], 1000, 0.01, th, x,
                     distance="l1", bank_scan="bf16")
    assert e.value.status == V.E_ARG
    ft50 = W.frame_times([1.0] * 50)
    with pytest.raises(V.VpetError) as e:
        V.bank_build([W.M_2TCM_IRR], W.box_array([W.M_2TCM_IRR]), 10, 1, W.grid(H, 50.0)[1], ft50, H)
    assert e.value.status == V.E_LIMIT


def test_infer_bank_full_size_sampled():
    """1,048,576 voxels against a 100,000-draw bank (30 frames, 0.1 % accepted),
    every voxel its own oracle curve plus noise, in the launch shape the
    benchmark times; 96 voxels spread over the volume (its ends, contraction
    block and voxel-chunk edges, random) against the oracle's bank form, each
    under the swap rule, none exempt."""
    import oracle as ora
    cfg = W.CFG_LARGE
    ft, cp = cfg.frame_times, cfg.input_fn()
    _, y = large_volume(cfg)
    sample = spread_sample(cfg.n_voxels, k=96, seed=4)
    models = list(cfg.models)
    boxes = cfg.box_array()
    th_g, x_g = V.bank_build(models, boxes, cfg.n_draws, cfg.infer_seed, cp, ft, H)
    res = V.infer_bank(torch.from_numpy(y).to(DEV), ft, H, cp.size, models, cfg.n_draws, cfg.accept_frac, th_g, x_g,
                       debug=True)
    torch.cuda.synchronize()
    sel = torch.from_numpy(sample).to(DEV)
    g_idx, g_mom, g_prob = (res[k][sel].cpu().numpy() for k in ("accept_idx", "moments", "model_prob"))
    assert torch.isfinite(res["model_prob"]).all()
    del res, th_g, x_g
    y_s = y[sample]
    o = ora.infer_bank(y_s, ft, cp, H, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed)
    th_o, x_o = ora.bank(models, boxes, cfg.n_draws, cfg.infer_seed, cp, H, ft)
    swaps = check_voxels(
        g_idx, g_mom, g_prob, o,
        dist_of=lambda j: bank_distances(ora, y_s[j], x_o, ft, H, cp.size),
        moments_of=lambda j, idx: ora.summarize_set(idx, models, boxes, cfg.n_draws, cfg.infer_seed, bank_theta=th_o),
        label="bank 1M")
    print(f"[bank full size] {len(sample)} sampled voxels, {swaps} with threshold swaps")
