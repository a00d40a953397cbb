"""ctypes binding of libvpetabc.so (include/vpet_abc.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  Device buffers are torch tensors on the current HIP device; the
work is enqueued on torch's current stream (or the one given).  There is no CPU
fallback: if the shared library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvpetabc.so")

OK, E_ARG, E_MODEL, E_GRID, E_HIP, E_NOMEM, E_LIMIT, E_IO = range(8)
M_1TCM, M_2TCM_IRR, M_2TCM_REV = 1, 2, 4
M_MRTM, M_LPNTPET = 8, 16  # reference-tissue models (input = reference TAC)
_ALL_MODELS = (M_1TCM, M_2TCM_IRR, M_2TCM_REV, M_MRTM, M_LPNTPET)
PSTRIDE = 8
MAX_ACCEPT = 3968

EXPORTED = ("vpet_abc_accept_count", "vpet_abc_simulate", "vpet_abc_infer", "vpet_abc_draws",
            "vpet_abc_bank_ld", "vpet_abc_bank_build", "vpet_abc_infer_bank", "vpet_abc_stream_bank",
            "vpet_abc_last_error", "vpet_abc_version", "vpet_proposal_init", "vpet_proposal_forward",
            "vpet_proposal_loss_grad", "vpet_proposal_train", "vpet_abc_infer_noalloc", "vpet_abc_bank_screen",
            "vpet_abc_infer_bank_learned", "vpet_abc_stream_bank_learned")
BANK_MAX_ACCEPT = 512
BANK_MAX_FRAMES = 48
PROPOSAL_NPARAM = 98912
PROPOSAL_NOUT = 96
PROPOSAL_MAX_FRAMES = 32


class VpetError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vpet_abc status {status}: {message}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("n_nodes", ctypes.c_int32), ("n_frames", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("decay_lambda", ctypes.c_double), ("weights", ctypes.c_void_p),
                ("weight_floor_frac", ctypes.c_float), ("distance", ctypes.c_int32),
                ("out_accept_idx", ctypes.c_void_p), ("out_accept_dist", ctypes.c_void_p),
                ("out_threshold", ctypes.c_void_p), ("voxel_offset", ctypes.c_int64),
                ("waves_per_voxel", ctypes.c_int32), ("bank_pilot", ctypes.c_int64),
                ("bank_scan", ctypes.c_int32), ("out_scan_ms", ctypes.POINTER(ctypes.c_float)),
                ("out_fallback_voxels", ctypes.POINTER(ctypes.c_int64)),
                ("proposal", ctypes.c_void_p), ("out_ess", ctypes.c_void_p),
                ("proposal_prior_share", ctypes.c_double), ("proposal_sd_scale", ctypes.c_double),
                ("accept_below", ctypes.c_void_p)]


class BankGroups(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("bins", ctypes.c_int32), ("group_voxels", ctypes.c_int32),
                ("prior_share", ctypes.c_double), ("sd_scale", ctypes.c_double), ("first_group", ctypes.c_int64),
                ("out_group", ctypes.c_void_p), ("out_bank_theta", ctypes.c_void_p),
                ("out_bank_logw", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, u32, u64, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    L.vpet_abc_accept_count.argtypes = [i64, f64, ctypes.POINTER(ctypes.c_int64)]
    L.vpet_abc_simulate.argtypes = [u32, P, i64, P, P, Grid, P, P]
    L.vpet_abc_infer.argtypes = [P, i64, P, P, Grid, u32, P, i64, f64, u64, P, P, ctypes.POINTER(Opts), P]
    L.vpet_abc_infer_noalloc.argtypes = L.vpet_abc_infer.argtypes
    L.vpet_abc_draws.argtypes = [u32, P, u64, P, P, P, i64, P, P, P]
    L.vpet_abc_bank_ld.argtypes = [ctypes.c_int32]
    L.vpet_abc_bank_ld.restype = ctypes.c_int
    L.vpet_abc_bank_build.argtypes = [u32, P, i64, u64, P, P, Grid, P, P, P]
    L.vpet_abc_infer_bank.argtypes = [P, i64, P, Grid, u32, i64, f64, P, P, P, P, ctypes.POINTER(Opts), P]
    L.vpet_abc_stream_bank.argtypes = [ctypes.c_char_p, i64, P, Grid, u32, i64, f64, P, P, i64, ctypes.c_char_p,
                                       ctypes.c_int32, i64, ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_int64), P]
    L.vpet_proposal_init.argtypes = [P, u64, P]
    L.vpet_proposal_forward.argtypes = [P, P, i64, ctypes.c_int32, P, P]
    L.vpet_proposal_loss_grad.argtypes = [P, P, P, i64, ctypes.c_int32, ctypes.c_int32, P, P, P]
    L.vpet_proposal_train.argtypes = [P, P, P, i64, P, ctypes.c_int32, ctypes.c_int32, f64, f64, i64, ctypes.c_int32,
                                      ctypes.c_float, u64, P, P]
    L.vpet_abc_last_error.restype = ctypes.c_char_p
    L.vpet_abc_version.restype = ctypes.c_int
    L.vpet_abc_bank_screen.argtypes = [P, i64, P, Grid, P, i64, ctypes.POINTER(Opts), P, P, P]
    L.vpet_abc_infer_bank_learned.argtypes = [P, i64, P, P, Grid, u32, P, P, ctypes.POINTER(BankGroups), i64, f64, u64,
                                              P, P, ctypes.POINTER(Opts), P]
    L.vpet_abc_stream_bank_learned.argtypes = [ctypes.c_char_p, i64, P, P, Grid, u32, P, P, ctypes.POINTER(BankGroups),
                                               i64, f64, u64, i64, ctypes.c_char_p, ctypes.c_int32, i64,
                                               ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_int64), P]
    for name in EXPORTED[:4] + EXPORTED[5:8] + EXPORTED[10:]:
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


def _check(status: int):
    if status != OK:
        raise VpetError(status, lib.vpet_abc_last_error().decode())


def model_mask(models) -> int:
    mask = 0
    for m in models:
        if m not in _ALL_MODELS:
            raise ValueError(f"unknown model {m}")
        mask |= int(m)
    if [m for m in _ALL_MODELS if mask & m] != list(models):
        raise ValueError("models must be distinct and listed in bit order (1TCM, IRR, REV, MRTM, lp-ntPET)")
    return mask


def accept_count(n_total: int, accept_frac: float) -> int:
    out = ctypes.c_int64()
    _check(lib.vpet_abc_accept_count(int(n_total), float(accept_frac), ctypes.byref(out)))
    return int(out.value)


def _host(a, dtype):
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 tensor on the GPU")
    return t


def simulate(model: int, theta, input_fn, frame_times, dt: float, out=None, stream=None):
    """Frame-averaged model TACs [n][F] (fp32) of parameter rows theta [n][8] (fp32, device)."""
    import torch
    theta = _dev_f32(theta, "theta")
    cp = _host(input_fn, np.float32)
    ft = _host(frame_times, np.float32)
    F = ft.size - 1
    n = theta.shape[0]
    if theta.dim() != 2 or theta.shape[1] != PSTRIDE:
        raise ValueError("theta must be [n][8]")
    if out is None:
        out = torch.empty((n, F), dtype=torch.float32, device=theta.device)
    grid = Grid(float(dt), cp.size, F)
    _check(lib.vpet_abc_simulate(int(model), _ptr(theta), n, cp.ctypes.data_as(ctypes.c_void_p),
                                 ft.ctypes.data_as(ctypes.c_void_p), grid, _ptr(out), _stream(stream)))
    return out


def infer(tacs, frame_times, input_fn, dt: float, models, prior_box, n_draws: int, accept_frac: float,
          seed: int, *, weights=None, weight_floor=0.0, decay_lambda=0.0, distance="l2", debug=False,
          voxel_offset=0, waves_per_voxel=0, proposal=None, prior_share=0.0, sd_scale=1.0, accept_below=None,
          out=None, stream=None, no_alloc=False) -> dict:
    """Voxelwise rejection ABC on observed TACs [V][F] (fp32, device).

    Returns a dict of device tensors: moments [V][M][8][2], model_prob [V][M]
    and, with debug=True, accept_idx [V][n], accept_dist [V][n], threshold [V].
    proposal: network outputs [V][96] (proposal_forward); the draws then come
    from each voxel's mixture (with a defensive prior share prior_share and
    every sd times sd_scale), the moments are importance-weighted and "ess"
    [V] is returned as well; accept_below [V] (fp32, device) then restricts the
    weighted summaries to the kept draws with distance <= accept_below[v] (ABC
    at a given threshold).  no_alloc=True calls vpet_abc_infer_noalloc
    (same results; the library allocates no device memory; pass `out` to keep
    this binding from allocating the output tensors).
    """
    import torch
    tacs = _dev_f32(tacs, "tacs")
    V, F = tacs.shape
    mask = model_mask(models)
    M = len(models)
    box = _host(prior_box, np.float64).reshape(M, PSTRIDE, 2)
    cp = _host(input_fn, np.float32)
    ft = _host(frame_times, np.float32)
    if ft.size != F + 1:
        raise ValueError("frame_times must have F + 1 entries")
    n = accept_count(M * int(n_draws), accept_frac)
    dev = tacs.device
    res = out if out is not None else {
        "moments": torch.empty((V, M, PSTRIDE, 2), dtype=torch.float32, device=dev),
        "model_prob": torch.empty((V, M), dtype=torch.float32, device=dev)}
    if debug and "accept_idx" not in res:
        res["accept_idx"] = torch.empty((V, n), dtype=torch.int32, device=dev)
        res["accept_dist"] = torch.empty((V, n), dtype=torch.float32, device=dev)
        res["threshold"] = torch.empty((V,), dtype=torch.float32, device=dev)
    o = Opts()
    o.decay_lambda = float(decay_lambda)
    if weights is not None:
        weights = _dev_f32(weights, "weights")
        if tuple(weights.shape) != (V, F):
            raise ValueError("weights must be [V][F]")
        o.weights = weights.data_ptr()
    o.weight_floor_frac = float(weight_floor)
    o.distance = {"l2": 0, "l1": 1}[distance]
    if debug:
        o.out_accept_idx = res["accept_idx"].data_ptr()
        o.out_accept_dist = res["accept_dist"].data_ptr()
        o.out_threshold = res["threshold"].data_ptr()
    o.voxel_offset = int(voxel_offset)
    o.waves_per_voxel = int(waves_per_voxel)
    if proposal is not None:
        proposal = _dev_f32(proposal, "proposal")
        if tuple(proposal.shape) != (V, PROPOSAL_NOUT):
            raise ValueError(f"proposal must be [V][{PROPOSAL_NOUT}]")
        o.proposal = proposal.data_ptr()
        o.proposal_prior_share = float(prior_share)
        o.proposal_sd_scale = float(sd_scale)
        if "ess" not in res:
            res["ess"] = torch.empty((V,), dtype=torch.float32, device=dev)
        o.out_ess = res["ess"].data_ptr()
    if accept_below is not None:
        accept_below = _dev_f32(accept_below, "accept_below")
        if tuple(accept_below.shape) != (V,):
            raise ValueError("accept_below must be [V]")
        o.accept_below = accept_below.data_ptr()
    grid = Grid(float(dt), cp.size, F)
    entry = lib.vpet_abc_infer_noalloc if no_alloc else lib.vpet_abc_infer
    _check(entry(_ptr(tacs), V, ft.ctypes.data_as(ctypes.c_void_p), cp.ctypes.data_as(ctypes.c_void_p),
                 grid, mask, box.ctypes.data_as(ctypes.c_void_p), int(n_draws), float(accept_frac),
                 int(seed) & ((1 << 64) - 1), _ptr(res["moments"]), _ptr(res["model_prob"]),
                 ctypes.byref(o), _stream(stream)))
    res["n"] = n
    return res


def infer_noalloc(*args, **kwargs) -> dict:
    """infer() through vpet_abc_infer_noalloc, the entry point that allocates no device memory."""
    return infer(*args, no_alloc=True, **kwargs)


def draws(models, prior_box, seed: int, voxel, draw, model_pos, stream=None):
    """Philox words [count][8] (int32 view of u32) and theta [count][8] for (voxel, draw, model_pos) triples."""
    import torch
    mask = model_mask(models)
    box = _host(prior_box, np.float64).reshape(len(models), PSTRIDE, 2)
    count = voxel.shape[0]
    for t, dt_, nm in ((voxel, torch.int64, "voxel"), (draw, torch.int64, "draw"), (model_pos, torch.int32, "model_pos")):
        if not (t.is_cuda and t.dtype == dt_ and t.is_contiguous() and t.shape[0] == count):
            raise TypeError(f"{nm} must be a contiguous {dt_} GPU tensor of length {count}")
    words = torch.empty((count, 8), dtype=torch.int32, device=voxel.device)
    theta = torch.empty((count, PSTRIDE), dtype=torch.float32, device=voxel.device)
    _check(lib.vpet_abc_draws(mask, box.ctypes.data_as(ctypes.c_void_p), int(seed) & ((1 << 64) - 1),
                              _ptr(voxel), _ptr(draw), _ptr(model_pos), count, _ptr(words), _ptr(theta),
                              _stream(stream)))
    return words, theta


def bank_build(models, prior_box, n_draws: int, seed: int, input_fn, frame_times, dt: float, device="cuda",
               stream=None):
    """Shared bank: parameters [M*n_draws][8] (fp32) and FP64 frame averages [M*n_draws][ld] (device)."""
    import torch
    mask = model_mask(models)
    M = len(models)
    box = _host(prior_box, np.float64).reshape(M, PSTRIDE, 2)
    cp = _host(input_fn, np.float32)
    ft = _host(frame_times, np.float32)
    F = ft.size - 1
    ld = int(lib.vpet_abc_bank_ld(F))
    n_tot = M * int(n_draws)
    theta = torch.empty((n_tot, PSTRIDE), dtype=torch.float32, device=device)
    x = torch.empty((n_tot, max(ld, 1)), dtype=torch.float64, device=device)
    _check(lib.vpet_abc_bank_build(mask, box.ctypes.data_as(ctypes.c_void_p), int(n_draws), int(seed) & ((1 << 64) - 1),
                                   cp.ctypes.data_as(ctypes.c_void_p), ft.ctypes.data_as(ctypes.c_void_p),
                                   Grid(float(dt), cp.size, F), _ptr(theta), _ptr(x), _stream(stream)))
    return theta, x


def infer_bank(tacs, frame_times, dt: float, n_nodes: int, models, n_draws: int, accept_frac: float, bank_theta,
               bank_x, *, weights=None, weight_floor=0.0, decay_lambda=0.0, distance="l2", debug=False,
               bank_pilot=0, bank_scan="auto", time_scan=False, out=None, stream=None) -> dict:
    """Rejection ABC of every voxel against one shared bank (see bank_build).

    time_scan: also return "scan_ms", the HIP-event time of the pair-screening
    kernel(s) (the call then waits for the stream)."""
    import torch
    tacs = _dev_f32(tacs, "tacs")
    V, F = tacs.shape
    mask = model_mask(models)
    M = len(models)
    ft = _host(frame_times, np.float32)
    if ft.size != F + 1:
        raise ValueError("frame_times must have F + 1 entries")
    if not (bank_x.dtype == torch.float64 and bank_theta.dtype == torch.float32):
        raise TypeError("bank_x must be float64 and bank_theta float32 (from bank_build)")
    n = accept_count(M * int(n_draws), accept_frac)
    dev = tacs.device
    res = out if out is not None else {
        "moments": torch.empty((V, M, PSTRIDE, 2), dtype=torch.float32, device=dev),
        "model_prob": torch.empty((V, M), dtype=torch.float32, device=dev)}
    if debug and "accept_idx" not in res:
        res["accept_idx"] = torch.empty((V, n), dtype=torch.int32, device=dev)
        res["accept_dist"] = torch.empty((V, n), dtype=torch.float32, device=dev)
        res["threshold"] = torch.empty((V,), dtype=torch.float32, device=dev)
    o = Opts()
    o.decay_lambda = float(decay_lambda)
    if weights is not None:
        weights = _dev_f32(weights, "weights")
        o.weights = weights.data_ptr()
    o.weight_floor_frac = float(weight_floor)
    o.distance = {"l2": 0, "l1": 1}[distance]
    if debug:
        o.out_accept_idx = res["accept_idx"].data_ptr()
        o.out_accept_dist = res["accept_dist"].data_ptr()
        o.out_threshold = res["threshold"].data_ptr()
    o.bank_pilot = int(bank_pilot)
    o.bank_scan = {"auto": 0, "f64": 1, "bf16": 2}[bank_scan]
    scan_ms = ctypes.c_float(0.0)
    n_fallback = ctypes.c_int64(0)
    if time_scan:
        o.out_scan_ms = ctypes.pointer(scan_ms)
    if debug:
        o.out_fallback_voxels = ctypes.pointer(n_fallback)
    _check(lib.vpet_abc_infer_bank(_ptr(tacs), V, ft.ctypes.data_as(ctypes.c_void_p), Grid(float(dt), int(n_nodes), F),
                                   mask, int(n_draws), float(accept_frac), _ptr(bank_theta), _ptr(bank_x),
                                   _ptr(res["moments"]), _ptr(res["model_prob"]), ctypes.byref(o), _stream(stream)))
    res["n"] = n
    if time_scan:
        res["scan_ms"] = float(scan_ms.value)
    if debug:
        res["fallback_voxels"] = int(n_fallback.value)
    return res


def infer_bank_learned(tacs, frame_times, input_fn, dt: float, models, prior_box, proposal, n_draws: int,
                       accept_frac: float, seed: int, *, dims=4, bins=4, group_voxels=256, prior_share=0.1,
                       sd_scale=1.0, weights=None, weight_floor=0.0, decay_lambda=0.0, distance="l2", debug=False,
                       bank_pilot=0, bank_scan="auto", time_scan=False, accept_below=None, return_bank=False,
                       first_group=0, out=None, stream=None) -> dict:
    """Shared-bank ABC with a learned proposal: voxels grouped by their network
    posterior (proposal [V][96] from proposal_forward with a head over `dims`
    parameters), one bank of n_draws rows per model per group drawn from the
    group's Gaussian mixed with the prior, rows weighted by prior / proposal.
    Returns moments, model_prob and ess (device); with debug, accept_idx
    (rows of the voxel's group bank), accept_dist, threshold and
    fallback_voxels; with return_bank, group [V], bank_theta [G][M n][8] and
    bank_logw [G][M n]; with time_scan, scan_ms."""
    import torch
    tacs = _dev_f32(tacs, "tacs")
    V, F = tacs.shape
    mask = model_mask(models)
    M = len(models)
    box = _host(prior_box, np.float64).reshape(M, PSTRIDE, 2)
    cp = _host(input_fn, np.float32)
    ft = _host(frame_times, np.float32)
    if ft.size != F + 1:
        raise ValueError("frame_times must have F + 1 entries")
    proposal = _dev_f32(proposal, "proposal")
    if tuple(proposal.shape) != (V, PROPOSAL_NOUT):
        raise ValueError(f"proposal must be [V][{PROPOSAL_NOUT}]")
    n = accept_count(M * int(n_draws), accept_frac)
    dev = tacs.device
    res = out if out is not None else {
        "moments": torch.empty((V, M, PSTRIDE, 2), dtype=torch.float32, device=dev),
        "model_prob": torch.empty((V, M), dtype=torch.float32, device=dev)}
    if "ess" not in res:
        res["ess"] = torch.empty((V,), dtype=torch.float32, device=dev)
    if debug and "accept_idx" not in res:
        res["accept_idx"] = torch.empty((V, n), dtype=torch.int32, device=dev)
        res["accept_dist"] = torch.empty((V, n), dtype=torch.float32, device=dev)
        res["threshold"] = torch.empty((V,), dtype=torch.float32, device=dev)
    gp = BankGroups()
    gp.dims, gp.bins, gp.group_voxels = int(dims), int(bins), int(group_voxels)
    gp.prior_share, gp.sd_scale = float(prior_share), float(sd_scale)
    gp.first_group = int(first_group)
    if return_bank:
        G = -(-V // int(group_voxels))
        res["group"] = torch.empty((V,), dtype=torch.int32, device=dev)
        res["bank_theta"] = torch.empty((G, M * int(n_draws), PSTRIDE), dtype=torch.float32, device=dev)
        res["bank_logw"] = torch.empty((G, M * int(n_draws)), dtype=torch.float64, device=dev)
        gp.out_group = res["group"].data_ptr()
        gp.out_bank_theta = res["bank_theta"].data_ptr()
        gp.out_bank_logw = res["bank_logw"].data_ptr()
    o = Opts()
    o.decay_lambda = float(decay_lambda)
    if weights is not None:
        weights = _dev_f32(weights, "weights")
        if tuple(weights.shape) != (V, F):
            raise ValueError("weights must be [V][F]")
        o.weights = weights.data_ptr()
    o.weight_floor_frac = float(weight_floor)
    o.distance = {"l2": 0, "l1": 1}[distance]
    if debug:
        o.out_accept_idx = res["accept_idx"].data_ptr()
        o.out_accept_dist = res["accept_dist"].data_ptr()
        o.out_threshold = res["threshold"].data_ptr()
    o.bank_pilot = int(bank_pilot)
    o.bank_scan = {"auto": 0, "f64": 1, "bf16": 2}[bank_scan]
    o.out_ess = res["ess"].data_ptr()
    if accept_below is not None:
        accept_below = _dev_f32(accept_below, "accept_below")
        if tuple(accept_below.shape) != (V,):
            raise ValueError("accept_below must be [V]")
        o.accept_below = accept_below.data_ptr()
    scan_ms = ctypes.c_float(0.0)
    n_fallback = ctypes.c_int64(0)
    if time_scan:
        o.out_scan_ms = ctypes.pointer(scan_ms)
    if debug:
        o.out_fallback_voxels = ctypes.pointer(n_fallback)
    _check(lib.vpet_abc_infer_bank_learned(_ptr(tacs), V, ft.ctypes.data_as(ctypes.c_void_p),
                                           cp.ctypes.data_as(ctypes.c_void_p), Grid(float(dt), cp.size, F), mask,
                                           box.ctypes.data_as(ctypes.c_void_p), _ptr(proposal), ctypes.byref(gp),
                                           int(n_draws), float(accept_frac), int(seed) & ((1 << 64) - 1),
                                           _ptr(res["moments"]), _ptr(res["model_prob"]), ctypes.byref(o),
                                           _stream(stream)))
    res["n"] = n
    if time_scan:
        res["scan_ms"] = float(scan_ms.value)
    if debug:
        res["fallback_voxels"] = int(n_fallback.value)
    return res


def bank_screen(tacs, frame_times, dt: float, n_nodes: int, bank_x, *, weights=None, weight_floor=0.0,
                decay_lambda=0.0, stream=None):
    """The BF16 contraction scan's computed S [V][N] (fp32) and a_v [V] (FP64) of
    every (voxel, bank row) pair, for checking the scan's error bound."""
    import torch
    tacs = _dev_f32(tacs, "tacs")
    V, F = tacs.shape
    ft = _host(frame_times, np.float32)
    if ft.size != F + 1:
        raise ValueError("frame_times must have F + 1 entries")
    if not (isinstance(bank_x, torch.Tensor) and bank_x.is_cuda and bank_x.dtype == torch.float64
            and bank_x.is_contiguous() and bank_x.dim() == 2 and bank_x.shape[1] == int(lib.vpet_abc_bank_ld(F))):
        raise TypeError("bank_x must be a contiguous float64 [N][bank_ld(F)] tensor on the GPU")
    N = bank_x.shape[0]
    o = Opts()
    o.decay_lambda = float(decay_lambda)
    o.weight_floor_frac = float(weight_floor)
    if weights is not None:
        weights = _dev_f32(weights, "weights")
        if tuple(weights.shape) != (V, F):
            raise ValueError("weights must be [V][F]")
        o.weights = weights.data_ptr()
    s = torch.empty((V, N), dtype=torch.float32, device=tacs.device)
    a = torch.empty((V,), dtype=torch.float64, device=tacs.device)
    _check(lib.vpet_abc_bank_screen(_ptr(tacs), V, ft.ctypes.data_as(ctypes.c_void_p), Grid(float(dt), int(n_nodes), F),
                                    _ptr(bank_x), N, ctypes.byref(o), _ptr(s), _ptr(a), _stream(stream)))
    return s, a


def stream_bank(tacs_path: str, n_voxels: int, frame_times, dt: float, n_nodes: int, models, n_draws: int,
                accept_frac: float, bank_theta, bank_x, out_prefix: str, *, chunk_voxels: int = 1 << 20,
                resume: bool = True, max_chunks: int = 0, weight_floor=0.0, decay_lambda=0.0, distance="l2",
                bank_pilot=0, bank_scan="auto", stream=None) -> int:
    """Shared-bank inference of a volume stored as raw fp32 [n_voxels][F] in
    tacs_path, streamed in chunks; outputs go to <out_prefix>.moments/.prob
    (see load_stream_outputs).  Returns the number of completed chunks."""
    import torch
    if not (bank_x.dtype == torch.float64 and bank_theta.dtype == torch.float32):
        raise TypeError("bank_x must be float64 and bank_theta float32 (from bank_build)")
    ft = _host(frame_times, np.float32)
    o = Opts()
    o.decay_lambda = float(decay_lambda)
    o.weight_floor_frac = float(weight_floor)
    o.distance = {"l2": 0, "l1": 1}[distance]
    o.bank_pilot = int(bank_pilot)
    o.bank_scan = {"auto": 0, "f64": 1, "bf16": 2}[bank_scan]
    done = ctypes.c_int64(0)
    _check(lib.vpet_abc_stream_bank(str(tacs_path).encode(), int(n_voxels), ft.ctypes.data_as(ctypes.c_void_p),
                                    Grid(float(dt), int(n_nodes), ft.size - 1), model_mask(models), int(n_draws),
                                    float(accept_frac), _ptr(bank_theta), _ptr(bank_x), int(chunk_voxels),
                                    str(out_prefix).encode(), int(bool(resume)), int(max_chunks), ctypes.byref(o),
                                    ctypes.byref(done), _stream(stream)))
    return int(done.value)


def stream_bank_learned(tacs_path: str, n_voxels: int, frame_times, input_fn, dt: float, models, prior_box, params,
                        n_draws: int, accept_frac: float, seed: int, out_prefix: str, *, dims=4, bins=4,
                        group_voxels=256, prior_share=0.1, sd_scale=1.0, chunk_voxels: int = 1 << 20,
                        resume: bool = True, max_chunks: int = 0, weight_floor=0.0, decay_lambda=0.0,
                        distance="l2", bank_pilot=0, bank_scan="auto", stream=None) -> int:
    """stream_bank with a learned proposal: per chunk the network (params) and
    infer_bank_learned; outputs as stream_bank.  Returns the completed chunks."""
    params = _params(params)
    ft = _host(frame_times, np.float32)
    cp = _host(input_fn, np.float32)
    M = len(models)
    box = _host(prior_box, np.float64).reshape(M, PSTRIDE, 2)
    gp = BankGroups()
    gp.dims, gp.bins, gp.group_voxels = int(dims), int(bins), int(group_voxels)
    gp.prior_share, gp.sd_scale = float(prior_share), float(sd_scale)
    o = Opts()
    o.decay_lambda = float(decay_lambda)
    o.weight_floor_frac = float(weight_floor)
    o.distance = {"l2": 0, "l1": 1}[distance]
    o.bank_pilot = int(bank_pilot)
    o.bank_scan = {"auto": 0, "f64": 1, "bf16": 2}[bank_scan]
    done = ctypes.c_int64(0)
    _check(lib.vpet_abc_stream_bank_learned(str(tacs_path).encode(), int(n_voxels), ft.ctypes.data_as(ctypes.c_void_p),
                                            cp.ctypes.data_as(ctypes.c_void_p), Grid(float(dt), cp.size, ft.size - 1),
                                            model_mask(models), box.ctypes.data_as(ctypes.c_void_p), _ptr(params),
                                            ctypes.byref(gp), int(n_draws), float(accept_frac),
                                            int(seed) & ((1 << 64) - 1), int(chunk_voxels), str(out_prefix).encode(),
                                            int(bool(resume)), int(max_chunks), ctypes.byref(o), ctypes.byref(done),
                                            _stream(stream)))
    return int(done.value)


def load_stream_outputs(out_prefix: str, n_voxels: int, n_models: int):
    """Read-only memory maps of a streamed run's moments [V][M][8][2] and
    model probabilities [V][M] (fp32)."""
    mom = np.memmap(str(out_prefix) + ".moments", dtype=np.float32, mode="r",
                    shape=(int(n_voxels), int(n_models), PSTRIDE, 2))
    prob = np.memmap(str(out_prefix) + ".prob", dtype=np.float32, mode="r", shape=(int(n_voxels), int(n_models)))
    return mom, prob


def proposal_init(seed: int, device="cuda", stream=None):
    """A freshly initialised parameter blob [PROPOSAL_NPARAM] (fp32, device)."""
    import torch
    p = torch.empty((PROPOSAL_NPARAM,), dtype=torch.float32, device=device)
    _check(lib.vpet_proposal_init(_ptr(p), int(seed) & ((1 << 64) - 1), _stream(stream)))
    return p


def _params(p):
    p = _dev_f32(p, "params")
    if p.numel() != PROPOSAL_NPARAM:
        raise ValueError(f"params must hold {PROPOSAL_NPARAM} floats")
    return p


def proposal_forward(params, tacs, out=None, stream=None):
    """Network outputs [V][96] (fp32, device) of TACs [V][F]."""
    import torch
    params, tacs = _params(params), _dev_f32(tacs, "tacs")
    V, F = tacs.shape
    if out is None:
        out = torch.empty((V, PROPOSAL_NOUT), dtype=torch.float32, device=tacs.device)
    _check(lib.vpet_proposal_forward(_ptr(params), _ptr(tacs), V, F, _ptr(out), _stream(stream)))
    return out


def proposal_loss_grad(params, tacs, theta, dims=4, stream=None):
    """(loss [1], grad [PROPOSAL_NPARAM]) device tensors of one batch:
    TACs [n][F] and parameter rows theta [n][8]; a head over `dims` (4 or 5)
    parameters."""
    import torch
    params, tacs, theta = _params(params), _dev_f32(tacs, "tacs"), _dev_f32(theta, "theta")
    n, F = tacs.shape
    if tuple(theta.shape) != (n, PSTRIDE):
        raise ValueError("theta must be [n][8]")
    g = torch.empty((PROPOSAL_NPARAM,), dtype=torch.float32, device=tacs.device)
    loss = torch.empty((1,), dtype=torch.float32, device=tacs.device)
    _check(lib.vpet_proposal_loss_grad(_ptr(params), _ptr(tacs), _ptr(theta), n, F, int(dims), _ptr(g), _ptr(loss),
                                       _stream(stream)))
    return loss, g


def proposal_train(params, bank_theta, bank_x, frame_times, *, steps: int, batch: int = 4096, lr: float = 5e-4,
                   noise_level: float = 0.1, decay_lambda: float = 0.0, seed: int = 0, dims: int = 4, stream=None):
    """Adam steps on params (in place) over a shared bank (irreversible 2TCM
    for dims = 4, reversible for dims = 5); returns the per-step batch losses
    (numpy, waits for the stream)."""
    import torch
    params = _params(params)
    if not (bank_x.dtype == torch.float64 and bank_theta.dtype == torch.float32):
        raise TypeError("bank_x must be float64 and bank_theta float32 (from bank_build)")
    ft = _host(frame_times, np.float32)
    losses = np.zeros(int(steps), dtype=np.float32)
    _check(lib.vpet_proposal_train(_ptr(params), _ptr(bank_theta), _ptr(bank_x), int(bank_theta.shape[0]),
                                   ft.ctypes.data_as(ctypes.c_void_p), ft.size - 1, int(dims), float(noise_level),
                                   float(decay_lambda), int(steps), int(batch), float(lr),
                                   int(seed) & ((1 << 64) - 1),
                                   losses.ctypes.data_as(ctypes.c_void_p) if steps > 0 else None, _stream(stream)))
    return losses


def version() -> int:
    return int(lib.vpet_abc_version())


DEFAULT_LAMBDA = math.log(2.0) / 109.8
