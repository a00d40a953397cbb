"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and rejects invalid requests with the documented status before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def V():
    import paper_2603_14859_amd as mod
    return mod


def test_exports_every_declared_symbol(V):
    hdr = open(os.path.join(ROOT, "include", "vpet_abc.h")).read()
    declared = set(re.findall(r"\b(vpet_(?:abc|proposal)_\w+)\s*\(", hdr))
    assert declared == set(V.EXPORTED)
    for name in declared:
        assert hasattr(V.lib, name)
    assert V.version() == 10000


def test_accept_count(V):
    import oracle
    for n_tot, p in [(2000, 0.01), (100000, 0.001), (10, 0.3), (3, 0.999), (7, 1.0), (10**9, 1e-7)]:
        assert V.accept_count(n_tot, p) == oracle.accept_count(n_tot, p)
    for n_tot, p in [(10, 0.05), (10, 0.0), (10, 1.5), (0, 0.5), (10, float("nan"))]:
        with pytest.raises(V.VpetError) as e:
            V.accept_count(n_tot, p)
        assert e.value.status == V.E_ARG


def _call_infer(V, *, model=2, ft=None, cp=None, dt=0.2, box=None, n_draws=100, p=0.1, V_=0, F=None, opts=None):
    ft = W.frame_times(W.SCHED_22x60) if ft is None else np.asarray(ft, dtype=np.float32)
    cp = W.grid(0.2, 60.0)[1] if cp is None else np.asarray(cp, dtype=np.float32)
    M = bin(model).count("1") if model else 1
    box = W.box_array([2] * M) if box is None else np.asarray(box, dtype=np.float64)
    F = ft.size - 1 if F is None else F
    grid = V._binding.Grid(dt, cp.size, F)
    st = V.lib.vpet_abc_infer(None, V_, ft.ctypes.data_as(ctypes.c_void_p), cp.ctypes.data_as(ctypes.c_void_p), grid,
                              model, box.ctypes.data_as(ctypes.c_void_p), n_draws, p, 1, None, None,
                              ctypes.byref(opts) if opts is not None else None, None)
    return st, V.lib.vpet_abc_last_error().decode()


def test_infer_validation_without_gpu(V):
    assert _call_infer(V)[0] == V.OK                      # V = 0: nothing to do
    assert _call_infer(V, model=0)[0] == V.E_MODEL
    assert _call_infer(V, model=8)[0] == V.E_MODEL
    assert _call_infer(V, p=0.0)[0] == V.E_ARG
    assert _call_infer(V, p=0.001)[0] == V.E_ARG          # n = 0
    assert _call_infer(V, n_draws=0)[0] == V.E_ARG
    assert _call_infer(V, n_draws=200000, p=0.5)[0] == V.E_LIMIT
    bad = W.frame_times(W.SCHED_22x60).copy()
    bad[3] += np.float32(0.05)
    assert _call_infer(V, ft=bad)[0] == V.E_GRID
    assert _call_infer(V, ft=np.array([0, 1, 1], np.float32), F=2)[0] == V.E_GRID
    assert _call_infer(V, ft=np.array([0, 1, 70], np.float32), F=2)[0] == V.E_GRID
    box = W.box_array([2])
    box[0, 0] = (0.5, 0.1)
    st, msg = _call_infer(V, box=box)
    assert st == V.E_ARG and "lo > hi" in msg
    box = W.box_array([2])
    box[0, 4] = (0.0, 1.0)
    assert _call_infer(V, box=box)[0] == V.E_ARG          # vB must stay below 1
    box = W.box_array([4])
    box[0, 2] = (0.0, 0.3)
    assert _call_infer(V, model=4, box=box)[0] == V.E_ARG  # reversible needs k3_lo > 0
    box = W.box_array([2])
    box[0, 1] = (0.0, 1.0)
    box[0, 2] = (0.0, 0.3)
    assert _call_infer(V, box=box)[0] == V.E_ARG          # 2TCM needs k2_lo + k3_lo > 0
    box = W.box_array([2])
    box[0, 1] = (-0.1, 1.0)
    assert _call_infer(V, box=box)[0] == V.E_ARG
    box = W.box_array([2])
    box[0, 0] = (0.0, np.inf)
    assert _call_infer(V, box=box)[0] == V.E_ARG
    o = V._binding.Opts()
    o.distance = 3
    assert _call_infer(V, opts=o)[0] == V.E_ARG
    o = V._binding.Opts()
    o.waves_per_voxel = 3
    assert _call_infer(V, opts=o)[0] == V.E_ARG
    o = V._binding.Opts()
    o.voxel_offset = 2**32 + 5
    assert _call_infer(V, opts=o)[0] == V.E_ARG
    assert _call_infer(V, dt=0.0)[0] == V.E_GRID
    cp = W.grid(0.2, 60.0)[1].copy()
    cp[4] = np.nan
    assert _call_infer(V, cp=cp)[0] == V.E_ARG


def test_simulate_and_draws_validation_without_gpu(V):
    ft = W.frame_times(W.SCHED_22x60)
    cp = W.grid(0.2, 60.0)[1]
    g = V._binding.Grid(0.2, cp.size, ft.size - 1)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert V.lib.vpet_abc_simulate(6, None, 10, P(cp), P(ft), g, None, None) == V.E_MODEL
    assert V.lib.vpet_abc_simulate(2, None, -1, P(cp), P(ft), g, None, None) == V.E_ARG
    assert V.lib.vpet_abc_simulate(2, None, 0, P(cp), P(ft), g, None, None) == V.OK
    g2 = V._binding.Grid(0.2, cp.size, 5)
    assert V.lib.vpet_abc_simulate(2, None, 0, P(cp), P(np.array([0, .2, .3, .4, .6, .8], np.float32)), g2, None,
                                   None) == V.E_GRID
    box = W.box_array([2])
    assert V.lib.vpet_abc_draws(0, P(box), 1, None, None, None, 5, None, None, None) == V.E_MODEL
    assert V.lib.vpet_abc_draws(2, P(box), 1, None, None, None, 0, None, None, None) == V.OK
    assert V.lib.vpet_abc_draws(2, P(box), 1, None, None, None, 5, None, None, None) == V.E_ARG
    assert V.lib.vpet_abc_last_error().decode() != ""


def test_bank_validation_without_gpu(V):
    ft = W.frame_times(W.SCHED_22x60)
    cp = W.grid(0.2, 60.0)[1]
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    g = V._binding.Grid(0.2, cp.size, ft.size - 1)
    box = W.box_array([2])
    assert V.lib.vpet_abc_bank_ld(22) == 24 and V.lib.vpet_abc_bank_ld(32) == 32 and V.lib.vpet_abc_bank_ld(0) == 0
    assert V.lib.vpet_abc_bank_build(0, P(box), 10, 1, P(cp), P(ft), g, None, None, None) == V.E_MODEL
    assert V.lib.vpet_abc_bank_build(2, P(box), 0, 1, P(cp), P(ft), g, None, None, None) == V.E_ARG
    assert V.lib.vpet_abc_bank_build(2, P(box), 10, 1, P(cp), P(ft), g, None, None, None) == V.E_ARG  # NULL outs
    ft40 = W.frame_times([1.0] * 50)
    g40 = V._binding.Grid(0.2, 251, 50)
    cp40 = W.grid(0.2, 50.0)[1]
    assert V.lib.vpet_abc_bank_build(2, P(box), 10, 1, P(cp40), P(ft40), g40, None, None, None) == V.E_LIMIT

    def ib(model=2, n_draws=1000, p=0.05, grid=g, frames=ft, V_=0, opts=None):
        return V.lib.vpet_abc_infer_bank(None, V_, P(frames), grid, model, n_draws, p, None, None, None, None,
                                         ctypes.byref(opts) if opts is not None else None, None)
    assert ib() == V.OK                                   # no voxels: nothing to do
    assert ib(model=0) == V.E_MODEL
    assert ib(p=0.9) == V.E_LIMIT                         # n = 900 > 512
    assert ib(p=0.0001) == V.E_ARG                        # n = 0
    bad = ft.copy()
    bad[2] += np.float32(0.07)
    assert ib(frames=bad) == V.E_GRID
    assert ib(grid=g40, frames=ft40) == V.E_LIMIT
    o = V._binding.Opts()
    o.bank_pilot = -1
    assert ib(opts=o) == V.E_ARG
    o = V._binding.Opts()
    o.bank_scan = 3
    assert ib(opts=o) == V.E_ARG                          # unknown scan
    o.bank_scan, o.distance = 2, 1
    assert ib(opts=o) == V.E_ARG                          # bf16 contraction is L2-only
    # reference-tissue models: no mixing with plasma-input models, valid tP box
    assert V.lib.vpet_abc_bank_build(2 | 8, P(W.box_array([2, 8])), 10, 1, P(cp), P(ft), g, None, None,
                                     None) == V.E_MODEL
    rbox = W.box_array([16])
    assert V.lib.vpet_abc_bank_build(16, P(rbox), 10, 1, P(cp), P(ft), g, None, None, None) == V.E_ARG  # NULL outs
    for slot, bad in ((5, (0.0, 70.0)), (5, (25.0, 70.0)), (6, (0.0, 4.0)), (2, (0.0, 0.2))):
        b2 = rbox.copy()
        b2[0, slot] = bad
        assert V.lib.vpet_abc_bank_build(16, P(b2), 10, 1, P(cp), P(ft), g, None, None, None) == V.E_ARG, slot
    assert V.lib.vpet_abc_infer(None, 0, P(ft), P(cp), g, 8, P(W.box_array([8])), 10, 0.5, 1, None, None, None,
                                None) == V.E_MODEL                # the per-voxel path does not run them
    assert ib(V_=3) == V.E_ARG                            # NULL device pointers


def test_stream_validation_without_gpu(V, tmp_path):
    ft = W.frame_times(W.SCHED_22x60)
    cp = W.grid(0.2, 60.0)[1]
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    g = V._binding.Grid(0.2, cp.size, ft.size - 1)
    fake = ctypes.c_void_p(256)  # bank pointers are only checked for NULL before the files
    path = tmp_path / "tacs.f32"
    np.ones((10, 22), dtype=np.float32).tofile(path)
    prefix = str(tmp_path / "out").encode()

    def sb(p=str(path).encode(), nv=10, resume=0, opts=None, chunk=4):
        return V.lib.vpet_abc_stream_bank(p, nv, P(ft), g, 2, 1000, 0.01, fake, fake, chunk, prefix, resume, 0,
                                          ctypes.byref(opts) if opts is not None else None, None, None)
    assert sb(p=str(tmp_path / "missing.f32").encode()) == V.E_IO
    assert sb(nv=11) == V.E_IO                            # file shorter than 11 x 22 values
    assert sb(chunk=0) == V.E_ARG
    o = V._binding.Opts()
    o.weights = 1234
    assert sb(opts=o) == V.E_ARG                          # no caller weights in streaming
    (tmp_path / "out.progress").write_text("vpet_abc_stream v1 voxels=99 frames=22 models=1 chunk=4 done=1\n")
    assert sb(resume=1) == V.E_ARG                        # progress of a run of another shape
    assert V.lib.vpet_abc_stream_bank(str(path).encode(), 10, P(ft), g, 0, 1000, 0.01, fake, fake, 4, prefix, 0, 0,
                                      None, None, None) == V.E_MODEL


def test_proposal_validation_without_gpu(V):
    """The learned-proposal entry points and the proposal option of
    vpet_abc_infer refuse bad requests before any device work."""
    L = V.lib
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert L.vpet_proposal_init(None, 1, None) == V.E_ARG
    assert L.vpet_proposal_forward(fake, fake, 10, 33, fake, None) == V.E_LIMIT
    assert L.vpet_proposal_forward(fake, fake, 10, 0, fake, None) == V.E_LIMIT
    assert L.vpet_proposal_forward(fake, fake, -1, 30, fake, None) == V.E_ARG
    assert L.vpet_proposal_forward(fake, fake, 0, 30, fake, None) == V.OK  # nothing to do
    assert L.vpet_proposal_forward(None, fake, 4, 30, fake, None) == V.E_ARG
    assert L.vpet_proposal_loss_grad(fake, fake, fake, 0, 30, 4, fake, fake, None) == V.E_ARG
    assert L.vpet_proposal_loss_grad(fake, fake, fake, (1 << 20) + 1, 30, 4, fake, fake, None) == V.E_ARG
    assert L.vpet_proposal_loss_grad(fake, fake, None, 8, 30, 4, fake, fake, None) == V.E_ARG
    assert L.vpet_proposal_loss_grad(fake, fake, fake, 8, 40, 4, fake, fake, None) == V.E_LIMIT
    assert L.vpet_proposal_loss_grad(fake, fake, fake, 8, 30, 3, fake, fake, None) == V.E_ARG
    ft = W.frame_times(W.SCHED_30x50)
    ftp = ft.ctypes.data_as(ctypes.c_void_p)

    def train(n_bank=1000, ft_=ftp, F=30, noise=0.1, lam=0.0, steps=5, batch=64, lr=1e-3, dims=4):
        return L.vpet_proposal_train(fake, fake, fake, n_bank, ft_, F, dims, noise, lam, steps, batch, lr, 1, None,
                                     None)
    assert train(n_bank=0) == V.E_ARG
    assert train(dims=6) == V.E_ARG
    assert train(steps=-1) == V.E_ARG
    assert train(batch=0) == V.E_ARG
    assert train(lr=0.0) == V.E_ARG
    assert train(lr=float("nan")) == V.E_ARG
    assert train(noise=-1.0) == V.E_ARG
    assert train(F=33) == V.E_LIMIT
    bad = ft.copy()
    bad[3] = bad[2]
    assert train(ft_=bad.ctypes.data_as(ctypes.c_void_p)) == V.E_GRID
    assert train(steps=0) == V.OK  # validated, nothing to do
    o = V._binding.Opts()
    o.proposal = 0x1000
    assert _call_infer(V, model=1, V_=1, box=W.box_array([1]), opts=o)[0] == V.E_MODEL
    assert _call_infer(V, model=6, V_=1, box=W.box_array([2, 4]), opts=o)[0] == V.E_MODEL
    o.proposal_prior_share = 1.5
    assert _call_infer(V, V_=1, opts=o)[0] == V.E_ARG
    o.proposal_prior_share = float("nan")
    assert _call_infer(V, V_=1, opts=o)[0] == V.E_ARG
    o.proposal_prior_share = 0.1
    o.proposal_sd_scale = -1.0
    assert _call_infer(V, V_=1, opts=o)[0] == V.E_ARG
    o.proposal_sd_scale = float("inf")
    assert _call_infer(V, V_=1, opts=o)[0] == V.E_ARG
    o2 = V._binding.Opts()
    o2.out_ess = 0x1000
    assert _call_infer(V, V_=1, opts=o2)[0] == V.E_ARG


def test_learned_bank_validation_without_gpu(V):
    """vpet_abc_infer_bank_learned refuses bad requests before any device work."""
    ft = W.frame_times(W.SCHED_30x50)
    cp = W.grid(0.2, 50.0)[1]
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    g = V._binding.Grid(0.2, cp.size, ft.size - 1)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first

    def lbank(model=2, dims=4, bins=4, gv=256, share=0.1, scale=1.0, n_draws=1000, p=0.05, V_=0, opts=None,
              groups=True):
        box = W.box_array([m for m in (1, 2, 4) if model & m] or [2])
        gp = V._binding.BankGroups()
        gp.dims, gp.bins, gp.group_voxels, gp.prior_share, gp.sd_scale = dims, bins, gv, share, scale
        return V.lib.vpet_abc_infer_bank_learned(None, V_, P(ft), P(cp), g, model, P(box), None,
                                                 ctypes.byref(gp) if groups else None, n_draws, p, 1, None, None,
                                                 ctypes.byref(opts) if opts is not None else None, None)
    assert lbank() == V.OK                                 # no voxels: nothing to do
    assert lbank(model=2 | 4, dims=5) == V.OK
    assert lbank(model=1) == V.E_MODEL                     # the 2TCMs only
    assert lbank(model=8) == V.E_MODEL
    assert lbank(groups=False) == V.E_ARG
    assert lbank(dims=3) == V.E_ARG
    assert lbank(bins=0) == V.E_ARG
    assert lbank(bins=9) == V.E_LIMIT                      # 9^4 cells > 4096
    assert lbank(gv=300) == V.E_ARG and lbank(gv=0) == V.E_ARG
    assert lbank(share=1.5) == V.E_ARG and lbank(scale=-1.0) == V.E_ARG
    assert lbank(p=0.9) == V.E_LIMIT                       # n = 900 > 512
    o = V._binding.Opts()
    o.proposal = 0x1000
    assert lbank(opts=o) == V.E_ARG                        # the proposal is an argument of its own
    o = V._binding.Opts()
    o.bank_scan, o.distance = 2, 1
    assert lbank(opts=o) == V.E_ARG                        # bf16 contraction is L2-only
    assert lbank(V_=3) == V.E_ARG                          # NULL device pointers
    # the prior bank form refuses the learned-proposal options
    o = V._binding.Opts()
    o.accept_below = 0x1000
    assert V.lib.vpet_abc_infer_bank(None, 0, P(ft), g, 2, 1000, 0.05, None, None, None, None, ctypes.byref(o),
                                     None) == V.E_ARG
    assert V.lib.vpet_abc_infer(None, 0, P(ft), P(cp), g, 2, P(W.box_array([2])), 10, 0.5, 1, None, None,
                                ctypes.byref(o), None) == V.E_ARG  # accept_below needs a proposal
    del fake
