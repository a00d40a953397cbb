"""Streaming of a volume stored in a file through the shared-bank form
(total-body scale, Sec. III-B2): the outputs equal those of one
vpet_abc_infer_bank call on the same data, chunk boundaries and a resumed run
included, and sampled streamed voxels equal the oracle's bank form."""
import numpy as np
import pytest

import workloads as W
from parity import bank_distances, check_voxels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2603_14859_amd as V  # noqa: E402

DEV = torch.device("cuda:0")


def _volume(cfg):
    import oracle as ora
    th, rev, eps = cfg.truth_mixture()
    ft, cp = cfg.frame_times, cfg.input_fn()
    clean = np.empty((cfg.n_voxels, ft.size - 1))
    thi = th[~rev].copy()
    thi[:, 3] = np.nan
    clean[~rev] = ora.simulate(W.M_2TCM_IRR, thi, cp, cfg.dt, ft)
    clean[rev] = ora.simulate(W.M_2TCM_REV, th[rev], cp, cfg.dt, ft)
    y = W.add_noise(clean, ft, eps)
    y[7, 3] = np.nan  # an invalid voxel inside the first chunk
    return y, rev


def test_stream_matches_one_call_and_resumes(tmp_path):
    cfg = W.CFG_TBPET_SMALL
    ft, cp = cfg.frame_times, cfg.input_fn()
    models, boxes = list(cfg.models), cfg.box_array()
    y, rev = _volume(cfg)
    path = tmp_path / "volume.f32"
    y.astype(np.float32).tofile(path)
    th_g, x_g = V.bank_build(models, boxes, cfg.n_draws, cfg.infer_seed, cp, ft, cfg.dt)
    ref = V.infer_bank(torch.from_numpy(y).to(DEV), ft, cfg.dt, cp.size, models, cfg.n_draws, cfg.accept_frac,
                       th_g, x_g, debug=True)
    torch.cuda.synchronize()
    ref_mom, ref_prob = ref["moments"].cpu().numpy(), ref["model_prob"].cpu().numpy()
    ref_idx = ref["accept_idx"].cpu().numpy()
    prefix = tmp_path / "run"
    args = (str(path), cfg.n_voxels, ft, cfg.dt, cp.size, models, cfg.n_draws, cfg.accept_frac, th_g, x_g,
            str(prefix))
    # interrupted after one chunk, then resumed; chunk 1024 leaves a ragged last chunk
    assert V.stream_bank(*args, chunk_voxels=1024, resume=False, max_chunks=1) == 1
    assert "done=1" in (tmp_path / "run.progress").read_text()
    assert V.stream_bank(*args, chunk_voxels=1024, resume=True) == 3
    assert "done=3" in (tmp_path / "run.progress").read_text()
    mom, prob = V.load_stream_outputs(str(prefix), cfg.n_voxels, len(models))
    assert np.array_equal(np.asarray(mom).view(np.uint32), ref_mom.view(np.uint32))
    assert np.array_equal(np.asarray(prob).view(np.uint32), ref_prob.view(np.uint32))
    assert np.isnan(prob[7]).all()
    # a completed run resumes to a no-op; a fresh run with another chunk size agrees
    assert V.stream_bank(*args, chunk_voxels=1024, resume=True) == 3
    assert V.stream_bank(*args, chunk_voxels=700, resume=False) == 5
    mom2, prob2 = V.load_stream_outputs(str(prefix), cfg.n_voxels, len(models))
    assert np.array_equal(np.asarray(mom2).view(np.uint32), ref_mom.view(np.uint32))
    # streamed voxels against the oracle's bank form: both sides of every chunk
    # boundary of both chunkings (1024 and 700), voxels written by the resumed
    # run, the invalid voxel and random ones.  The streamed outputs equal the
    # in-memory call's bit for bit (above), so that call's accepted sets are
    # the streamed ones.
    import oracle as ora
    sample = sorted({0, 7, 1023, 1024, 2047, 2048, 2999, 699, 700, 1399, 1400, 2099, 2100, 2799, 2800}
                    | set(np.random.default_rng(5).choice(cfg.n_voxels, 17, replace=False).tolist()))
    sample = np.array(sample)
    y_s = y[sample]
    o = ora.infer_bank(y_s, ft, cp, cfg.dt, models, boxes, cfg.n_draws, cfg.accept_frac, cfg.infer_seed)
    th_o, x_o = ora.bank(models, boxes, cfg.n_draws, cfg.infer_seed, cp, cfg.dt, ft)
    valid = sample != 7
    assert np.isnan(np.asarray(mom2)[7]).all() and (ref_idx[7] == -1).all()
    vs = sample[valid]
    swaps = check_voxels(
        ref_idx[vs], np.asarray(mom2)[vs], np.asarray(prob2)[vs],
        {k: o[k][valid] for k in ("accept_idx", "threshold", "moments", "model_prob")},
        dist_of=lambda j: bank_distances(ora, y[vs[j]], x_o, ft, cfg.dt, cp.size),
        moments_of=lambda j, idx: ora.summarize_set(idx, models, boxes, cfg.n_draws, cfg.infer_seed, bank_theta=th_o),
        label="stream")
    print(f"[stream vs oracle] {vs.size} streamed voxels, {swaps} with threshold swaps")
    # the reversible half prefers the reversible model on average
    p_rev = np.asarray(prob2)[:, 1]
    ok = ~np.isnan(p_rev)
    assert p_rev[ok & rev].mean() > p_rev[ok & ~rev].mean()


def test_stream_learned_matches_chunked_calls_resumes_and_matches_oracle(tmp_path):
    """Streaming with a learned proposal: each chunk's outputs equal those of
    one vpet_abc_infer_bank_learned call on that chunk (network outputs from
    vpet_proposal_forward, groups numbered on from the previous chunks'),
    across an interrupted and resumed run; streamed voxels on both sides of
    the chunk boundaries against the oracle (with the same network outputs,
    which the forward-pass parity tests check separately).  A progress file
    of a prior-bank run is not resumed by a learned run."""
    import oracle.learned_bank as lb
    cfg = W.CFG_TBPET_SMALL
    ft, cp = cfg.frame_times, cfg.input_fn()
    models, boxes = list(cfg.models), cfg.box_array()
    y, rev = _volume(cfg)
    path = tmp_path / "volume.f32"
    y.astype(np.float32).tofile(path)
    params = V.proposal_init(3)
    gk = dict(dims=5, bins=2, group_voxels=256, prior_share=0.2, sd_scale=1.5)
    n_draws, p, seed, chunk = 2000, 0.01, 17, 1024
    prefix = tmp_path / "learned"
    args = (str(path), cfg.n_voxels, ft, cp, cfg.dt, models, boxes, params, n_draws, p, seed, str(prefix))
    assert V.stream_bank_learned(*args, chunk_voxels=chunk, resume=False, max_chunks=2, **gk) == 2
    assert V.stream_bank_learned(*args, chunk_voxels=chunk, resume=True, **gk) == 3
    text = (tmp_path / "learned.progress").read_text()
    assert text.startswith("vpet_abc_stream_learned") and "done=3" in text
    mom, prob = V.load_stream_outputs(str(prefix), cfg.n_voxels, len(models))
    y_d = torch.from_numpy(y).to(DEV)
    outs = {}
    for c in range(3):
        sl = slice(c * chunk, min(cfg.n_voxels, (c + 1) * chunk))
        o_c = V.proposal_forward(params, y_d[sl].contiguous())
        r = V.infer_bank_learned(y_d[sl].contiguous(), ft, cp, cfg.dt, models, boxes, o_c, n_draws, p, seed,
                                 debug=True, first_group=c * (chunk // 256), **gk)
        torch.cuda.synchronize()
        assert np.array_equal(np.asarray(mom[sl]).view(np.uint32), r["moments"].cpu().numpy().view(np.uint32))
        assert np.array_equal(np.asarray(prob[sl]).view(np.uint32), r["model_prob"].cpu().numpy().view(np.uint32))
        outs[c] = (o_c.cpu().numpy().astype(np.float64), r["accept_idx"].cpu().numpy())
    assert np.isnan(prob[7]).all()
    # oracle on voxels both sides of the chunk boundaries
    for c, local in ((0, [0, 1, 1022, 1023]), (1, [0, 1, 1023]), (2, [0, 500, cfg.n_voxels - 2049])):
        sl = slice(c * chunk, min(cfg.n_voxels, (c + 1) * chunk))
        o_c, idx = outs[c]
        ref = lb.infer_bank_learned(y[sl], ft, cp, cfg.dt, models, boxes, o_c, n_draws, p, seed, voxels=local,
                                    first_group=c * (chunk // 256), **gk)
        for k, v in enumerate(local):
            a_g, a_o = set(idx[v].tolist()), set(ref["accept_idx"][k].tolist())
            if a_g != a_o:
                d, h = ref["distances"][k], ref["threshold"][k]
                assert all(abs(d[q] - h) <= 1e-5 * h for q in a_g ^ a_o), (c, v)
                continue
            gm = np.asarray(mom[sl])[v].astype(np.float64)
            ok = ~np.isnan(ref["moments"][k])
            assert np.array_equal(np.isnan(gm), ~ok), (c, v)
            assert np.allclose(gm[ok], ref["moments"][k][ok], rtol=1e-5, atol=1e-7), (c, v)
            assert np.allclose(np.asarray(prob[sl])[v], ref["model_prob"][k], atol=1e-6), (c, v)
    # a prior-bank run's progress is not continued by a learned run
    (tmp_path / "learned.progress").write_text(
        f"vpet_abc_stream v1 voxels={cfg.n_voxels} frames={ft.size - 1} models=2 chunk={chunk} done=1\n")
    with pytest.raises(V.VpetError):
        V.stream_bank_learned(*args, chunk_voxels=chunk, resume=True, **gk)
