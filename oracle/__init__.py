"""FP64 CPU oracle for voxelwise ABC rejection (vPET-ABC, arXiv 2603.14859).

TEST INFRASTRUCTURE ONLY: the plain reference that the HIP library is checked
against.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2603_14859_amd``) and neither imports the other.

The arithmetic lives in ``vpet_oracle.c`` (plain C, FP64, one voxel and one draw
at a time, a library sort for the selection).  This module only loads the
shared object and marshals numpy arrays.  See the header of ``vpet_oracle.c``
for the paper passages each step follows and the readings adopted where the
paper is silent.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vpet_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libvpet_oracle.so")

M_1TCM = 1
M_2TCM_IRR = 2
M_2TCM_REV = 4
M_MRTM = 8      # reference-tissue models: the input is the reference TAC C_r
M_LPNTPET = 16
NSLOT = 8
SLOT = {"K1": 0, "k2": 1, "k3": 2, "k4": 3, "vB": 4, "Ki": 5}
SLOT_REF = {"R1": 0, "k2": 1, "k2a": 2, "gamma": 3, "tD": 4, "tP": 5, "alpha": 6, "BP": 7}
DEFAULT_LAMBDA = math.log(2.0) / 109.8  # 18F, min^-1 (Sec. III-A1)
DEFAULT_FLOOR = 0.01

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, u32, u64, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        L.ora_philox_batch.argtypes = [P, i64, u64, P]
        L.ora_draw_batch.argtypes = [P, P, u64, P, P, P, i64, u32, P, P, P]
        L.ora_step_coeffs.argtypes = [f64, f64, P, P, P]
        L.ora_convolve_exp.argtypes = [f64, P, i32, f64, P]
        L.ora_simulate_nodes.argtypes = [u32, P, P, i32, f64, P]
        L.ora_frame_average.argtypes = [P, P, i32, P]
        L.ora_simulate.argtypes = [u32, P, i64, P, i32, f64, P, i32, P]
        L.ora_simulate_f64.argtypes = [u32, P, i64, P, i32, f64, P, i32, P]
        L.ora_weights.argtypes = [P, P, i32, f64, f64, f64, P]
        L.ora_accept_count.argtypes = [i64, f64]
        L.ora_accept_count.restype = i64
        L.ora_infer.argtypes = [P, i64, i32, P, i32, f64, P, P, i32, P, i64, f64, u64, i64, f64, f64,
                                i32, P, i32, P, P, P, P, P]
        L.ora_infer.restype = i64
        L.ora_voxel_distances.argtypes = [P, i32, P, i32, f64, P, P, i32, P, i64, u64, i64, f64, f64,
                                          i32, P, P]
        L.ora_bank.argtypes = [P, i32, P, i64, u64, P, i32, f64, P, i32, P, P]
        L.ora_infer_bank.argtypes = [P, i64, i32, P, i32, f64, P, P, i32, P, i64, f64, u64, f64, f64, i32, P, i32,
                                     P, P, P, P, P]
        L.ora_infer_bank.restype = i64
        L.ora_summarize_set.argtypes = [P, i64, P, i32, P, i64, u64, u64, ctypes.c_uint32, P, P, P]
        L.ora_gamma_variate.argtypes = [f64, f64, f64, f64]
        L.ora_gamma_variate.restype = f64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# Grid and frames (reading: frame bounds lie on the nodes t_k = k * dt).
# --------------------------------------------------------------------------
def frame_nodes(frame_times, dt: float, n_nodes: int) -> np.ndarray:
    """Node index of every frame bound; raises if a bound is off the grid."""
    ft = np.asarray(frame_times, dtype=np.float32).astype(np.float64)
    h = float(np.float32(dt))
    kf = np.rint(ft / h).astype(np.int64)
    if np.any(np.abs(kf * h - ft) > 1e-6 * np.maximum(1.0, np.abs(ft))):
        raise ValueError("frame bound not on the time grid")
    if np.any(np.diff(kf) <= 0) or kf[0] < 0 or kf[-1] > n_nodes - 1:
        raise ValueError("frame bounds must increase and lie within the grid")
    return kf.astype(np.int32)


def accept_count(n_tot: int, p: float) -> int:
    return int(lib().ora_accept_count(int(n_tot), float(p)))


# --------------------------------------------------------------------------
# Draws (Alg. 1 lines 1-2, Philox4x32-10).
# --------------------------------------------------------------------------
def philox(counters, seed: int) -> np.ndarray:
    c = _c(counters, np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    lib().ora_philox_batch(_p(c), c.shape[0], int(seed), _p(out))
    return out


def draws(models, boxes, seed, v, i, m, stream=0):
    """Philox words [n][8], unit floats [n][8] and fp32 theta [n][8]."""
    mo = _c(models, np.uint32)
    bx = _c(boxes, np.float64).reshape(len(mo), NSLOT, 2)
    vv, ii, mm = _c(v, np.int64), _c(i, np.int64), _c(m, np.int32)
    n = vv.shape[0]
    theta = np.full((n, NSLOT), np.nan, dtype=np.float32)
    words = np.zeros((n, 8), dtype=np.uint32)
    u = np.full((n, 8), np.nan, dtype=np.float32)
    lib().ora_draw_batch(_p(mo), _p(bx), int(seed), _p(vv), _p(ii), _p(mm), n, int(stream),
                         _p(theta), _p(words), _p(u))
    return words, u, theta


# --------------------------------------------------------------------------
# Forward model (Eq. (1)-(2); reading R2 for the discretisation).
# --------------------------------------------------------------------------
def gamma_variate(t: float, tD: float, tP: float, alpha: float) -> float:
    """lp-ntPET activation g(t) (0 up to tD, peak 1 at tP)."""
    return float(lib().ora_gamma_variate(float(t), float(tD), float(tP), float(alpha)))


def step_coeffs(beta: float, h: float):
    e, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().ora_step_coeffs(float(beta), float(h), ctypes.byref(e), ctypes.byref(a), ctypes.byref(b))
    return e.value, a.value, b.value


def convolve_exp(beta: float, cp, h: float) -> np.ndarray:
    c = _c(cp, np.float64)
    out = np.empty_like(c)
    lib().ora_convolve_exp(float(beta), _p(c), c.shape[0] - 1, float(h), _p(out))
    return out


def simulate_nodes(model: int, theta, cp, h: float) -> np.ndarray:
    th = _c(theta, np.float64).reshape(NSLOT)
    c = _c(cp, np.float64)
    out = np.empty_like(c)
    lib().ora_simulate_nodes(int(model), _p(th), _p(c), c.shape[0] - 1, float(h), _p(out))
    return out


def frame_average(nodes, kf) -> np.ndarray:
    nd = _c(nodes, np.float64)
    k = _c(kf, np.int32)
    out = np.empty(k.shape[0] - 1, dtype=np.float64)
    lib().ora_frame_average(_p(nd), _p(k), k.shape[0] - 1, _p(out))
    return out


def simulate(model: int, theta, input_fn, dt: float, frame_times) -> np.ndarray:
    """Frame-averaged TACs [n][F] (FP64) of fp32 parameter rows theta[n][8]."""
    cp = _c(np.asarray(input_fn, dtype=np.float32), np.float64)
    kf = frame_nodes(frame_times, dt, cp.shape[0])
    h = float(np.float32(dt))
    if np.asarray(theta).dtype == np.float64:
        th = _c(theta, np.float64).reshape(-1, NSLOT)
        out = np.empty((th.shape[0], kf.shape[0] - 1), dtype=np.float64)
        lib().ora_simulate_f64(int(model), _p(th), th.shape[0], _p(cp), cp.shape[0] - 1, h, _p(kf),
                               kf.shape[0] - 1, _p(out))
        return out
    th = _c(theta, np.float32).reshape(-1, NSLOT)
    out = np.empty((th.shape[0], kf.shape[0] - 1), dtype=np.float64)
    lib().ora_simulate(int(model), _p(th), th.shape[0], _p(cp), cp.shape[0] - 1, h, _p(kf),
                       kf.shape[0] - 1, _p(out))
    return out


def weights(y, frame_times, dt, n_nodes, lam=DEFAULT_LAMBDA, floor=DEFAULT_FLOOR) -> np.ndarray:
    yy = _c(y, np.float32)
    kf = frame_nodes(frame_times, dt, n_nodes)
    w = np.empty(yy.shape[0], dtype=np.float64)
    lib().ora_weights(_p(yy), _p(kf), kf.shape[0] - 1, float(np.float32(dt)), float(lam), float(floor),
                      _p(w))
    return w


# --------------------------------------------------------------------------
# Fixed-budget rejection ABC (Alg. 1) and posterior summaries.
# --------------------------------------------------------------------------
def infer(tacs, frame_times, input_fn, dt, models, boxes, n_draws, accept_frac, seed,
          voxel_offset=0, lam=DEFAULT_LAMBDA, floor=DEFAULT_FLOOR, l1=False, weights=None,
          nthreads=0) -> dict:
    y = _c(tacs, np.float32)
    V, F = y.shape
    cp = _c(input_fn, np.float32)
    kf = frame_nodes(frame_times, dt, cp.shape[0])
    if kf.shape[0] - 1 != F:
        raise ValueError("tacs and frame_times disagree on the frame count")
    mo = _c(models, np.uint32)
    M = mo.shape[0]
    bx = _c(boxes, np.float64).reshape(M, NSLOT, 2)
    n = accept_count(M * int(n_draws), accept_frac)
    if n == 0:
        raise ValueError("accept count n = floor(N p) must be >= 1")
    acc_g = np.empty((V, n), dtype=np.int32)
    acc_d = np.empty((V, n), dtype=np.float64)
    thr = np.empty((V, 2), dtype=np.float64)
    mom = np.empty((V, M, NSLOT, 2), dtype=np.float64)
    pr = np.empty((V, M), dtype=np.float64)
    w = None if weights is None else _c(weights, np.float32)
    got = lib().ora_infer(_p(y), V, F, _p(cp), cp.shape[0] - 1, float(np.float32(dt)), _p(kf), _p(mo), M,
                          _p(bx), int(n_draws), float(accept_frac), int(seed), int(voxel_offset),
                          float(lam), float(floor), int(bool(l1)),
                          None if w is None else _p(w), int(nthreads),
                          _p(acc_g), _p(acc_d), _p(thr), _p(mom), _p(pr))
    assert got == n
    return {"n": n, "accept_idx": acc_g, "accept_dist": acc_d, "threshold": thr[:, 0],
            "next_dist": thr[:, 1], "moments": mom, "model_prob": pr}


def voxel_distances(y_v, frame_times, input_fn, dt, models, boxes, n_draws, seed, v_global,
                    lam=DEFAULT_LAMBDA, floor=DEFAULT_FLOOR, l1=False, weights_v=None) -> np.ndarray:
    yv = _c(y_v, np.float32)
    cp = _c(input_fn, np.float32)
    kf = frame_nodes(frame_times, dt, cp.shape[0])
    mo = _c(models, np.uint32)
    M = mo.shape[0]
    bx = _c(boxes, np.float64).reshape(M, NSLOT, 2)
    out = np.empty(M * int(n_draws), dtype=np.float64)
    w = None if weights_v is None else _c(weights_v, np.float32)
    lib().ora_voxel_distances(_p(yv), yv.shape[0], _p(cp), cp.shape[0] - 1, float(np.float32(dt)), _p(kf),
                              _p(mo), M, _p(bx), int(n_draws), int(seed), int(v_global), float(lam),
                              float(floor), int(bool(l1)), None if w is None else _p(w), _p(out))
    return out


def summarize_set(idx, models, boxes, n_draws, seed, v_global=0, bank_theta=None):
    """The oracle's FP64 summaries (moments [M][8][2], probabilities [M]) of an
    explicit accepted set of global draw indices: regenerated per-voxel draws of
    voxel v_global, or rows of the shared bank's parameters bank_theta."""
    ii = _c(idx, np.int32)
    mo = _c(models, np.uint32)
    M = mo.shape[0]
    bx = _c(boxes, np.float64).reshape(M, NSLOT, 2)
    th = None if bank_theta is None else _c(bank_theta, np.float32)
    mom = np.empty((M, NSLOT, 2), dtype=np.float64)
    pr = np.empty(M, dtype=np.float64)
    lib().ora_summarize_set(_p(ii), ii.shape[0], _p(mo), M, _p(bx), int(n_draws), int(seed), int(v_global),
                            0 if th is None else 1, None if th is None else _p(th), _p(mom), _p(pr))
    return mom, pr


# --------------------------------------------------------------------------
# Shared-bank form (Alg. 1 as printed): one bank of prior draws and curves
# for all voxels; bank draw i of list position m uses the Philox counter
# (i, 0, 1, m << 16 | blk).
# --------------------------------------------------------------------------
def bank(models, boxes, n_draws, seed, input_fn, dt, frame_times):
    """Bank parameters [M*n_draws][8] (fp32) and frame-averaged curves [M*n_draws][F] (FP64)."""
    mo = _c(models, np.uint32)
    M = mo.shape[0]
    bx = _c(boxes, np.float64).reshape(M, NSLOT, 2)
    cp = _c(input_fn, np.float32)
    kf = frame_nodes(frame_times, dt, cp.shape[0])
    F = kf.shape[0] - 1
    n_tot = M * int(n_draws)
    th = np.empty((n_tot, NSLOT), dtype=np.float32)
    x = np.empty((n_tot, F), dtype=np.float64)
    L = lib()
    L.ora_bank(_p(mo), M, _p(bx), int(n_draws), int(seed), _p(cp), cp.shape[0] - 1, float(np.float32(dt)), _p(kf), F,
               _p(th), _p(x))
    return th, x


def infer_bank(tacs, frame_times, input_fn, dt, models, boxes, n_draws, accept_frac, seed, lam=DEFAULT_LAMBDA,
               floor=DEFAULT_FLOOR, l1=False, weights=None, nthreads=0) -> dict:
    y = _c(tacs, np.float32)
    V, F = y.shape
    cp = _c(input_fn, np.float32)
    kf = frame_nodes(frame_times, dt, cp.shape[0])
    if kf.shape[0] - 1 != F:
        raise ValueError("tacs and frame_times disagree on the frame count")
    mo = _c(models, np.uint32)
    M = mo.shape[0]
    bx = _c(boxes, np.float64).reshape(M, NSLOT, 2)
    n = accept_count(M * int(n_draws), accept_frac)
    if n == 0:
        raise ValueError("accept count n = floor(N p) must be >= 1")
    acc_g = np.empty((V, n), dtype=np.int32)
    acc_d = np.empty((V, n), dtype=np.float64)
    thr = np.empty((V, 2), dtype=np.float64)
    mom = np.empty((V, M, NSLOT, 2), dtype=np.float64)
    pr = np.empty((V, M), dtype=np.float64)
    w = None if weights is None else _c(weights, np.float32)
    got = lib().ora_infer_bank(_p(y), V, F, _p(cp), cp.shape[0] - 1, float(np.float32(dt)), _p(kf), _p(mo), M, _p(bx),
                               int(n_draws), float(accept_frac), int(seed), float(lam), float(floor), int(bool(l1)),
                               None if w is None else _p(w), int(nthreads), _p(acc_g), _p(acc_d), _p(thr), _p(mom),
                               _p(pr))
    assert got == n
    return {"n": n, "accept_idx": acc_g, "accept_dist": acc_d, "threshold": thr[:, 0], "next_dist": thr[:, 1],
            "moments": mom, "model_prob": pr}
