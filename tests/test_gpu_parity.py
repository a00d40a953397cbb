"""GPU parity: the HIP library against the FP64 oracle on identical seeded inputs.

All calls go through the C ABI (ctypes binding).  Inputs come from the
`workloads` generators; observed TACs are made noise-free by the oracle's
forward model and then noised, so no input or expected value comes from the
GPU path.
"""
import numpy as np
import pytest

import workloads as W
from parity import (MEAN_RTOL, TAC_RTOL, check_voxels, compare_sets, large_volume, oracle_moments_of,
                    spread_sample, tac_rel_err)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU-only hosts
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2603_14859_amd as V  # noqa: E402  (fails loudly if the library is missing)

DEV = torch.device("cuda:0")
H = 0.2


def _inputs(sched=W.SCHED_22x60, n_vox=64, model=W.M_2TCM_IRR, seed=2603014859, level=0.05):
    import oracle as ora
    ft = W.frame_times(sched)
    _, cp = W.grid(H, float(np.sum(sched)))
    rng = np.random.default_rng(seed)
    box = W.box_array([model])[0]
    th = W.true_params(rng, n_vox, model, box)
    clean = ora.simulate(model, th, cp, H, ft)
    y = W.add_noise(clean, ft, rng.standard_normal(clean.shape), level=level)
    return ft, cp, y


def _gpu_infer(y, ft, cp, models, boxes, n_draws, p, seed, **kw):
    res = V.infer(torch.from_numpy(y).to(DEV), ft, cp, H, models, boxes, n_draws, p, seed, debug=True, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in res.items()}


def _check_infer(ora, y, ft, cp, models, boxes, n_draws, p, seed, voxel_offset=0, l1=False, weights=None,
                 wpv=0, strict_means=True):
    g = _gpu_infer(y, ft, cp, models, boxes, n_draws, p, seed, voxel_offset=voxel_offset,
                   distance="l1" if l1 else "l2", waves_per_voxel=wpv,
                   weights=None if weights is None else torch.from_numpy(weights).to(DEV))
    o = ora.infer(y, ft, cp, H, models, boxes, n_draws, p, seed, voxel_offset=voxel_offset, l1=l1,
                  weights=weights, nthreads=0)
    assert g["n"] == o["n"]
    nvox, swaps = compare_sets(ora, g["accept_idx"], o, y, ft, cp, H, models, boxes, n_draws, seed,
                               voxel_offset=voxel_offset, l1=l1, weights=weights)
    print(f"[parity] V={y.shape[0]} n={o['n']} voxels with boundary swaps: {nvox} ({len(swaps)} draws)")
    for v in range(y.shape[0]):
        same = set(g["accept_idx"][v].tolist()) == set(o["accept_idx"][v].tolist())
        if same:
            ref_mom, ref_prob = o["moments"][v], o["model_prob"][v]
        else:
            ref_mom, ref_prob = oracle_moments_of(ora, list(models), boxes, seed, v + voxel_offset,
                                                  g["accept_idx"][v], n_draws)
        gm = g["moments"][v].astype(np.float64)
        assert np.array_equal(np.isnan(gm), np.isnan(ref_mom)), f"voxel {v}: NaN pattern differs"
        ok = ~np.isnan(ref_mom)
        rt = 1e-5 if strict_means else MEAN_RTOL
        assert np.allclose(gm[..., 0][ok[..., 0]], ref_mom[..., 0][ok[..., 0]], rtol=rt, atol=1e-7), f"voxel {v} means"
        assert np.allclose(gm[..., 1][ok[..., 1]], ref_mom[..., 1][ok[..., 1]], rtol=1e-4, atol=1e-9), f"voxel {v} vars"
        assert np.allclose(g["model_prob"][v], ref_prob, rtol=0, atol=1e-7, equal_nan=True)
        # the accepted distances agree with the oracle's to fp32 rounding
        if same:
            assert np.allclose(np.sort(g["accept_dist"][v]), np.sort(o["accept_dist"][v]), rtol=1e-6, equal_nan=True)
    return g, o


# ---------------------------------------------------------------------------
# A1: draws bit-exact
# ---------------------------------------------------------------------------
def test_draws_bitexact():
    import oracle as ora
    models = [W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV]
    boxes = W.box_array(models)
    boxes[2, 1] = (0.013, 1.7)
    rng = np.random.default_rng(5)
    n = 8192
    v = rng.integers(0, 2**32, n)
    i = rng.integers(0, 2**32, n)
    m = rng.integers(0, 3, n).astype(np.int32)
    v[:3], i[:3] = [0, 2**32 - 1, 5], [0, 2**32 - 1, 7]
    for seed in (0, 14859, 2**64 - 1):
        w_g, th_g = V.draws(models, boxes, seed, torch.from_numpy(v.astype(np.int64)).to(DEV),
                            torch.from_numpy(i.astype(np.int64)).to(DEV), torch.from_numpy(m).to(DEV))
        w_o, _, th_o = ora.draws(models, boxes, seed, v, i, m)
        assert np.array_equal(w_g.cpu().numpy().view(np.uint32), w_o)
        assert np.array_equal(th_g.cpu().numpy().view(np.uint32), th_o.view(np.uint32))


# ---------------------------------------------------------------------------
# A2-A4: simulated TACs within 1e-5
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("model", [W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV])
@pytest.mark.parametrize("sched", ["22x60", "30x50", "offset"])
def test_simulate_parity(model, sched):
    import oracle as ora
    durations = {"22x60": W.SCHED_22x60, "30x50": W.SCHED_30x50, "offset": [0.2, 0.4, 1.0, 3.0, 5.4]}[sched]
    ft = W.frame_times(durations)
    t_end = float(np.sum(durations))
    if sched == "offset":   # first frame starts after t = 0, grid longer than the last frame
        ft = (ft + np.float32(1.4)).astype(np.float32)
        t_end += 3.0
    _, cp = W.grid(H, t_end)
    box = W.box_array([model])[0]
    if model == W.M_1TCM:
        box[1] = (0.0, 1.0)         # includes a zero rate
    rng = np.random.default_rng(model * 7 + len(durations))
    n = 60_000
    th = W.true_params(rng, n, model, box)
    # corners of the prior box (slowest / fastest rates, extreme blood fraction)
    slots = W.SLOTS[model]
    corners = np.array(np.meshgrid(*[[0, 1]] * len(slots))).reshape(len(slots), -1).T
    for r, c in enumerate(corners):
        for s, b in zip(slots, c):
            th[r, s] = np.float32(box[s][b])
    if model == W.M_2TCM_REV:
        th[-1000:, 3] = np.float32(0.0)                     # k4 = 0: a zero eigenvalue
        th[-2000:-1000, 3] = rng.uniform(0, 1e-7, 1000).astype(np.float32)
    got = V.simulate(model, torch.from_numpy(th).to(DEV), cp, ft, H).cpu().numpy()
    want = ora.simulate(model, th, cp, H, ft)
    err = tac_rel_err(got, want)
    print(f"[simulate] model={model} sched={sched} max rel err {err.max():.3e}")
    assert err.max() <= TAC_RTOL


# Rates up to 6/min put the step exponent x = rate * 0.2 min well above 0.3,
# where a wavefront leaves the short series for the general set-up (expm1 and
# the divided difference); the slow draws at the front keep whole wavefronts on
# the series, so both paths run in one launch.
FAST = {W.M_1TCM: {1: (0.01, 6.0)}, W.M_2TCM_IRR: {1: (0.01, 4.0), 2: (0.001, 2.0)},
        W.M_2TCM_REV: {1: (0.01, 4.0), 2: (0.001, 2.0), 3: (0.0, 1.0)}}


def _fast_box(model):
    box = W.box_array([model])[0]
    for s, lohi in FAST[model].items():
        box[s] = lohi
    return box


@pytest.mark.parametrize("model", [W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV])
def test_simulate_parity_fast_rates(model):
    import oracle as ora
    ft = W.frame_times(W.SCHED_30x50)
    _, cp = W.grid(H, float(np.sum(W.SCHED_30x50)))
    box = _fast_box(model)
    rng = np.random.default_rng(model + 40)
    th = W.true_params(rng, 20_000, model, box)
    th[:4096, 1] = np.float32(0.05)  # 64 wavefronts of slow draws: the series path
    if model != W.M_1TCM:
        th[:4096, 2] = np.float32(0.01)
    if model == W.M_2TCM_REV:
        th[:4096, 3] = np.float32(0.01)
    got = V.simulate(model, torch.from_numpy(th).to(DEV), cp, ft, H).cpu().numpy()
    want = ora.simulate(model, th, cp, H, ft)
    err = tac_rel_err(got, want)
    print(f"[simulate fast rates] model={model} max rel err {err.max():.3e}")
    assert err.max() <= TAC_RTOL


@pytest.mark.parametrize("models", [(W.M_2TCM_IRR,), (W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV)])
def test_infer_parity_fast_rates(models):
    import oracle as ora
    ft, cp, y = _inputs(W.SCHED_30x50, 24, model=W.M_2TCM_IRR, seed=19)
    boxes = np.stack([_fast_box(m) for m in models])
    _check_infer(ora, y, ft, cp, list(models), boxes, 1200, 0.02, 31)


# ---------------------------------------------------------------------------
# A0-A6 end to end: the small configuration at full size
# ---------------------------------------------------------------------------
def test_infer_parity_1024_voxels_22_frames():
    import oracle as ora
    cfg = W.CFG_SMALL
    ft, cp, y = _inputs(cfg.durations, cfg.n_voxels)
    models = [W.M_2TCM_IRR]
    boxes = W.box_array(models)
    _check_infer(ora, y, ft, cp, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed)


@pytest.mark.parametrize("models", [(W.M_2TCM_IRR, W.M_2TCM_REV), (W.M_1TCM, W.M_2TCM_IRR),
                                    (W.M_1TCM, W.M_2TCM_IRR, W.M_2TCM_REV)])
def test_infer_parity_model_selection(models):
    import oracle as ora
    ft, cp, y = _inputs(W.SCHED_30x50, 48, model=W.M_2TCM_REV, seed=11)
    boxes = W.box_array(list(models))
    _check_infer(ora, y, ft, cp, list(models), boxes, 1500, 0.01, 77)


def test_infer_parity_l1_and_caller_weights():
    import oracle as ora
    ft, cp, y = _inputs(W.SCHED_22x60, 40, seed=3)
    models = [W.M_2TCM_IRR]
    boxes = W.box_array(models)
    _check_infer(ora, y, ft, cp, models, boxes, 1000, 0.02, 5, l1=True)
    w = np.random.default_rng(2).uniform(0.2, 3.0, y.shape).astype(np.float32)
    w[3, 4], w[7, 0], w[9, 2] = -1.0, np.inf, 0.0  # invalid, invalid, allowed
    g, _ = _check_infer(ora, y, ft, cp, models, boxes, 1000, 0.02, 5, weights=w)
    assert np.isnan(g["moments"][[3, 7]]).all() and np.isfinite(g["moments"][9, 0, 5, 0])


@pytest.mark.parametrize("n_draws,p", [(1, 1.0), (77, 0.05), (1000, 1.0), (1984, 1.0), (333, 0.003)])
def test_infer_edge_sizes(n_draws, p):
    import oracle as ora
    ft, cp, y = _inputs(W.SCHED_22x60, 9, seed=n_draws)
    models = [W.M_2TCM_IRR, W.M_2TCM_REV]
    boxes = W.box_array(models)
    _check_infer(ora, y, ft, cp, models, boxes, n_draws, p, 123, voxel_offset=1000)


def test_infer_ties_nan_voxels_and_offsets():
    import oracle as ora
    ft, cp, y = _inputs(W.SCHED_22x60, 12, seed=4)
    y[3, 5] = np.nan
    y[7] = 0.0
    models = [W.M_2TCM_IRR]
    boxes = W.box_array(models)
    g, o = _check_infer(ora, y, ft, cp, models, boxes, 500, 0.04, 9, voxel_offset=77)
    for v in (3, 7):
        assert np.isnan(g["moments"][v]).all() and np.isnan(g["model_prob"][v]).all()
        assert (g["accept_idx"][v] == -1).all()
    # a degenerate prior: every distance ties, so the lowest indices win
    th = (0.4, 0.2, 0.05, 0.0, 0.04)
    dbox = np.zeros((1, 8, 2))
    for s in range(5):
        dbox[0, s] = (th[s], th[s])
    g = _gpu_infer(y[:2], ft, cp, models, dbox, 700, 0.1, 3)
    assert np.array_equal(g["accept_idx"], np.tile(np.arange(70), (2, 1)))


# n = 36, then n = 256 and 257 on either side of the size up to which the
# block merge sorts only each wavefront's first n keys
@pytest.mark.parametrize("n_draws,p", [(900, 0.02), (1280, 0.1), (1285, 0.1)])
def test_infer_deterministic_across_launch_shapes(n_draws, p):
    ft, cp, y = _inputs(W.SCHED_22x60, 33, seed=8)
    models = [W.M_2TCM_IRR, W.M_2TCM_REV]
    boxes = W.box_array(models)
    outs = [_gpu_infer(y, ft, cp, models, boxes, n_draws, p, 4, waves_per_voxel=w) for w in (1, 2, 4, 4)]
    for o in outs[1:]:
        for k in ("accept_idx", "accept_dist", "threshold", "moments", "model_prob"):
            assert np.array_equal(o[k], outs[0][k], equal_nan=True), k


def test_infer_zero_voxels_and_errors():
    t = torch.empty((0, 22), dtype=torch.float32, device=DEV)
    ft = W.frame_times(W.SCHED_22x60)
    _, cp = W.grid(H, 60.0)
    res = V.infer(t, ft, cp, H, [W.M_2TCM_IRR], W.box_array([W.M_2TCM_IRR]), 100, 0.1, 1)
    assert res["moments"].shape == (0, 1, 8, 2)
    y = torch.ones((2, 22), dtype=torch.float32, device=DEV)
    with pytest.raises(V.VpetError) as e:
        V.infer(y, ft, cp, H, [W.M_2TCM_IRR], W.box_array([W.M_2TCM_IRR]), 100_000, 0.05, 1)
    assert e.value.status == V.E_LIMIT


# ---------------------------------------------------------------------------
# Full size of the large configuration, in the launch shape the benchmark times:
# sampled voxels against the oracle.
# ---------------------------------------------------------------------------
def test_infer_full_size_large_config_sampled():
    """1,048,576 voxels x 100,000 per-voxel draws (30 frames, 0.1 % accepted),
    every voxel its own oracle curve plus noise; 96 voxels spread over the
    volume (its ends, block and chunk edges, random) against the oracle, each
    one under the swap rule, none exempt."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle as ora
    cfg = W.CFG_LARGE
    ft, cp = cfg.frame_times, cfg.input_fn()
    _, y = large_volume(cfg)
    sample = spread_sample(cfg.n_voxels, k=96)
    models = list(cfg.models)
    boxes = cfg.box_array()
    res = V.infer(torch.from_numpy(y).to(DEV), ft, cp, H, models, boxes, cfg.n_draws, cfg.accept_frac,
                  cfg.infer_seed, debug=True)
    torch.cuda.synchronize()
    sel = torch.from_numpy(sample).to(DEV)
    g_idx, g_mom, g_prob = (res[k][sel].cpu().numpy() for k in ("accept_idx", "moments", "model_prob"))
    assert torch.isfinite(res["model_prob"]).all()
    assert torch.isfinite(res["moments"][:, 0, [0, 1, 2, 4, 5], 0]).all()
    del res

    def one(v):  # the oracle on one voxel at its global index (ctypes releases the GIL)
        return ora.infer(y[v:v + 1], ft, cp, H, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed,
                         voxel_offset=int(v), nthreads=1)

    with ThreadPoolExecutor(8) as ex:
        outs = list(ex.map(one, sample))
    o = {k: np.concatenate([r[k] for r in outs]) for k in ("accept_idx", "threshold", "moments", "model_prob")}
    swaps = check_voxels(
        g_idx, g_mom, g_prob, o,
        dist_of=lambda j: ora.voxel_distances(y[sample[j]], ft, cp, H, models, boxes, cfg.n_draws,
                                              cfg.infer_seed, int(sample[j])),
        moments_of=lambda j, idx: ora.summarize_set(idx, models, boxes, cfg.n_draws, cfg.infer_seed,
                                                    v_global=int(sample[j])),
        label="per-voxel 1M")
    print(f"[full size] {len(sample)} sampled voxels, {swaps} with threshold swaps")
