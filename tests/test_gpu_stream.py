"""Streaming of a volume stored in a file through the shared-bank form
(total-body scale, Sec. III-B2): the outputs equal those of one
vpet_abc_infer_bank call on the same data, chunk boundaries and a resumed run
included."""
import numpy as np
import pytest

import workloads as W

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
                       th_g, x_g)
    torch.cuda.synchronize()
    ref_mom, ref_prob = ref["moments"].cpu().numpy(), ref["model_prob"].cpu().numpy()
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
    # the reversible half prefers the reversible model on average
    p_rev = np.asarray(prob2)[:, 1]
    ok = ~np.isnan(p_rev)
    assert p_rev[ok & rev].mean() > p_rev[ok & ~rev].mean()
