"""GPU parity of the reference-tissue models, MRTM and lp-ntPET (Sec. II-A2,
Eq. (3)-(4)), against the oracle, through the C ABI: draws (with the relative
tP box), forward model, shared bank, and model selection in the shared-bank
form."""
import numpy as np
import pytest

import workloads as W
from parity import THRESH_RTOL, bank_distances, check_voxels, spread_sample

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2603_14859_amd as V  # noqa: E402

DEV = torch.device("cuda:0")
MODELS = [W.M_MRTM, W.M_LPNTPET]


def _observed(cfg, n, seed_shift=0):
    """Noisy reference-tissue TACs of the config (half activated) via the oracle."""
    import oracle as ora
    th, active, eps = cfg.truth_reference(n)
    ft, cr = cfg.frame_times, cfg.input_fn()
    clean = np.empty((n, ft.size - 1))
    a = np.nonzero(active)[0]
    z = np.nonzero(~active)[0]
    if a.size:
        clean[a] = ora.simulate(W.M_LPNTPET, th[a], cr, cfg.dt, ft)
    if z.size:
        clean[z] = ora.simulate(W.M_MRTM, th[z], cr, cfg.dt, ft)
    return W.add_noise(clean, ft, eps, lam=cfg.decay_lambda), active


def test_reference_draws_bit_exact():
    import oracle as ora
    boxes = W.box_array(MODELS)
    rng = np.random.default_rng(3)
    n = 20000
    v = rng.integers(0, 2**32, n)
    i = rng.integers(0, 2**32, n)
    m = rng.integers(0, 2, n).astype(np.int32)
    words_o, _, th_o = ora.draws(np.array(MODELS, dtype=np.uint32), boxes, 77, v, i, m)
    words_g, th_g = V.draws(MODELS, boxes, 77, torch.from_numpy(v).to(DEV), torch.from_numpy(i).to(DEV),
                            torch.from_numpy(m).to(DEV))
    assert np.array_equal(words_g.cpu().numpy().view(np.uint32), words_o)
    assert np.array_equal(th_g.cpu().numpy().view(np.uint32), th_o.view(np.uint32))
    lp = m == 1
    assert np.all(th_o[lp, 5] >= th_o[lp, 4] + 1.0 - 1e-4) and np.all(th_o[lp, 5] <= 70.0)


@pytest.mark.parametrize("model", [W.M_MRTM, W.M_LPNTPET])
def test_reference_simulate_matches_oracle(model):
    import oracle as ora
    cfg = W.CFG_LPNT_SMALL
    ft, cr = cfg.frame_times, cfg.input_fn()
    box = W.box_array([model])
    rng = np.random.default_rng(11)
    n = 3000
    _, _, th = ora.draws(np.array([model], dtype=np.uint32), box, 5, rng.integers(0, 2**32, n),
                         rng.integers(0, 2**32, n), np.zeros(n, dtype=np.int32))
    # box corners: fastest/slowest rates, earliest/latest activation
    corner = th[:4].copy()
    corner[0, :3] = box[0, :3, 1]
    corner[1, :3] = box[0, :3, 0]
    if model == W.M_LPNTPET:
        corner[2, 3:7] = [0.5, 20.0, 21.0, 4.0]
        corner[3, 3:7] = [0.5, 50.0, 70.0, 0.25]
    th = np.vstack([corner, th])
    got = V.simulate(model, torch.from_numpy(th).to(DEV), cr, ft, cfg.dt).cpu().numpy()
    ref = ora.simulate(model, th, cr, cfg.dt, ft)
    err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
    assert err.max() < 1e-6, err.max()  # fp32 output of an FP64 computation


def test_reference_bank_build_matches_oracle():
    import oracle as ora
    cfg = W.CFG_LPNT_SMALL
    ft, cr = cfg.frame_times, cfg.input_fn()
    boxes = W.box_array(MODELS)
    th_g, x_g = V.bank_build(MODELS, boxes, 4000, 21, cr, ft, cfg.dt)
    th_o, x_o = ora.bank(MODELS, boxes, 4000, 21, cr, cfg.dt, ft)
    assert np.array_equal(th_g.cpu().numpy().view(np.uint32), th_o.view(np.uint32))
    F = ft.size - 1
    xg = x_g.cpu().numpy()
    assert xg.shape[1] == 40
    err = np.abs(xg[:, :F] - x_o).max(axis=1) / np.abs(x_o).max(axis=1)
    assert err.max() < 1e-11, err.max()


def _moments_of(th_bank, idx, n_draws, M):
    """FP64 per-model summaries of an explicit accepted set (canonical slots,
    BP_ND = k2/k2a - 1 in slot 7)."""
    t = th_bank[np.asarray(idx)].astype(np.float64)
    t[:, 7] = t[:, 1] / t[:, 2] - 1.0
    mm = np.asarray(idx) // n_draws
    mom = np.full((M, 8, 2), np.nan)
    prob = np.zeros(M)
    for k in range(M):
        sel = t[mm == k]
        prob[k] = sel.shape[0] / len(idx)
        used = [0, 1, 2, 7] if k == 0 else list(range(8))
        if sel.shape[0]:
            mom[k, used, 0] = sel[:, used].mean(axis=0)
            mom[k, used, 1] = sel[:, used].var(axis=0, ddof=1) if sel.shape[0] > 1 else 0.0
    return mom, prob


@pytest.mark.parametrize("scan", ["f64", "bf16"])
def test_reference_model_selection_parity(scan):
    import oracle as ora
    cfg = W.CFG_LPNT_SMALL
    ft, cr = cfg.frame_times, cfg.input_fn()
    boxes = W.box_array(MODELS)
    y, active = _observed(cfg, cfg.n_voxels)
    th_g, x_g = V.bank_build(MODELS, boxes, cfg.n_draws, cfg.infer_seed, cr, ft, cfg.dt)
    res = V.infer_bank(torch.from_numpy(y).to(DEV), ft, cfg.dt, cr.size, MODELS, cfg.n_draws, cfg.accept_frac,
                       th_g, x_g, decay_lambda=cfg.decay_lambda, debug=True, bank_scan=scan)
    torch.cuda.synchronize()
    g = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()}
    o = ora.infer_bank(y, ft, cr, cfg.dt, MODELS, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                       lam=cfg.decay_lambda)
    th_o, x_o = ora.bank(MODELS, boxes, cfg.n_draws, cfg.infer_seed, cr, cfg.dt, ft)
    assert g["n"] == o["n"] == 40
    swaps = 0
    for v in range(y.shape[0]):
        a_g, a_o = set(g["accept_idx"][v].tolist()), set(o["accept_idx"][v].tolist())
        if a_g != a_o:
            w = ora.weights(y[v], ft, cfg.dt, cr.size, lam=cfg.decay_lambda)
            d = (w * (y[v].astype(np.float64) - x_o) ** 2).sum(1)
            h = o["threshold"][v]
            for gg in a_g ^ a_o:
                assert abs(d[gg] - h) <= THRESH_RTOL * h, f"voxel {v}: draw {gg} swapped far from the threshold"
            swaps += 1
            ref_mom, ref_prob = _moments_of(th_o, g["accept_idx"][v], cfg.n_draws, 2)
        else:
            ref_mom, ref_prob = o["moments"][v], o["model_prob"][v]
        gm = g["moments"][v].astype(np.float64)
        assert np.array_equal(np.isnan(gm), np.isnan(ref_mom)), f"voxel {v}: NaN pattern"
        ok = ~np.isnan(ref_mom)
        assert np.allclose(gm[ok], ref_mom[ok], rtol=1e-5, atol=1e-6), f"voxel {v}: moments"
        assert np.allclose(g["model_prob"][v], ref_prob, atol=1e-7)
    print(f"[reference parity] scan={scan} V={y.shape[0]} swaps={swaps} fallbacks={g['fallback_voxels']}")
    p_lp = g["model_prob"][:, 1]
    assert p_lp[active].mean() > p_lp[~active].mean() + 0.1, (p_lp[active].mean(), p_lp[~active].mean())


def test_reference_models_refused_by_per_voxel_path_and_mixing():
    cfg = W.CFG_LPNT_SMALL
    ft, cr = cfg.frame_times, cfg.input_fn()
    y = torch.ones((4, ft.size - 1), device=DEV)
    with pytest.raises(V.VpetError) as e:
        V.infer(y, ft, cr, cfg.dt, [W.M_MRTM], W.box_array([W.M_MRTM]), 100, 0.1, 1)
    assert e.value.status == V.E_MODEL
    with pytest.raises(V.VpetError) as e:
        V.bank_build([W.M_2TCM_IRR, W.M_MRTM], W.box_array([W.M_2TCM_IRR, W.M_MRTM]), 100, 1, cr, ft, cfg.dt)
    assert e.value.status == V.E_MODEL


def test_reference_full_size_sampled():
    """1,556,480 voxels (128 x 128 x 95), 40 frames / 90 min, every voxel its
    own curve (half activated), against one bank of 200k MRTM + 200k lp-ntPET
    draws, 0.1 % accepted (n = 400); 64 voxels spread over the volume (its
    ends, contraction block and voxel-chunk edges, random) against the
    oracle's bank form, each under the swap rule, none exempt."""
    import oracle as ora
    cfg = W.CFG_LPNT
    ft, cr = cfg.frame_times, cfg.input_fn()
    boxes = W.box_array(MODELS)
    y, active = _observed(cfg, cfg.n_voxels)
    sample = spread_sample(cfg.n_voxels, k=64, seed=8, edges=(256, 131072))
    th_g, x_g = V.bank_build(MODELS, boxes, cfg.n_draws, cfg.infer_seed, cr, ft, cfg.dt)
    res = V.infer_bank(torch.from_numpy(y).to(DEV), ft, cfg.dt, cr.size, MODELS, cfg.n_draws, cfg.accept_frac,
                       th_g, x_g, decay_lambda=cfg.decay_lambda, debug=True)
    torch.cuda.synchronize()
    s_t = torch.from_numpy(sample).to(DEV)
    g_idx, g_mom, g_prob = (res[k][s_t].cpu().numpy() for k in ("accept_idx", "moments", "model_prob"))
    p_lp = res["model_prob"][:, 1].cpu().numpy()
    del res, th_g, x_g
    y_s = y[sample]
    o = ora.infer_bank(y_s, ft, cr, cfg.dt, MODELS, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                       lam=cfg.decay_lambda)
    assert o["n"] == 400
    th_o, x_o = ora.bank(MODELS, boxes, cfg.n_draws, cfg.infer_seed, cr, cfg.dt, ft)
    swaps = check_voxels(
        g_idx, g_mom, g_prob, o,
        dist_of=lambda j: bank_distances(ora, y_s[j], x_o, ft, cfg.dt, cr.size, lam=cfg.decay_lambda),
        moments_of=lambda j, idx: ora.summarize_set(idx, MODELS, boxes, cfg.n_draws, cfg.infer_seed, bank_theta=th_o),
        mean_atol=1e-6, label="lp-ntPET/MRTM 1.56M")
    # model selection over the whole volume: activated voxels prefer lp-ntPET far more often
    ok = np.isfinite(p_lp)
    sens, fpr = np.mean(p_lp[ok & active] > 0.5), np.mean(p_lp[ok & ~active] > 0.5)
    print(f"[reference full size] {len(sample)} sampled voxels, {swaps} with threshold swaps; "
          f"P(lp-ntPET) > 1/2 for {sens:.3f} of activated and {fpr:.3f} of null voxels")
    assert sens > 0.5 and fpr < 0.1
