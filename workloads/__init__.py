"""Seeded synthetic inputs for voxelwise ABC rejection (vPET-ABC, arXiv 2603.14859).

This module generates the *inputs* that both the GPU library and the CPU oracle
consume: the plasma input function sampled on the time grid, frame schedules,
prior boxes, "true" kinetic parameters and standard-normal noise, plus the
additive noise model that turns a noise-free TAC into an observed one.  It holds
none of the method's arithmetic (no sampling of the method's draws, no forward
simulation, no discrepancy, no selection): noise-free TACs are produced by the
caller with whichever forward model it is allowed to use.

The paper's datasets (its simulated TAC sets and clinical scans) are not
available; these seeded synthetic inputs stand in for them with the paper's
shapes and distributions:

* Input function: Feng's three-exponential plasma model (Sec. III-A1) with fixed
  parameters inside the paper's ranges, rescaled to kBq/mL and minutes.
* Noise: y = C + sqrt(level * C * exp(lambda t) / dt) * N(0, 1) with
  lambda = ln 2 / 109.8 min (18F) and level = 0.05 (kBq/mL units; the paper's
  l = 7 in Bq/mL gives 7^2 = 49 Bq ~ 0.05 kBq).
* True parameters: uniform over the prior box, as the paper draws its simulated
  parameters uniformly from literature ranges.
* Reference-tissue configurations (MRTM vs lp-ntPET, Sec. II-A2): the input is
  a reference-region TAC, the closed-form one-tissue response
  K1' exp(-k2' t) * C_a(t) to the same Feng input (K1' = 0.1 /min, k2' = 0.2
  /min: not in the paper), 11C decay (lambda = ln 2 / 20.4 min); half of the
  voxels carry an activation (lp-ntPET truth), half none (MRTM truth).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

M_1TCM = 1
M_2TCM_IRR = 2
M_2TCM_REV = 4
M_MRTM = 8
M_LPNTPET = 16
NSLOT = 8
SLOTS = {M_1TCM: (0, 1, 4), M_2TCM_IRR: (0, 1, 2, 4), M_2TCM_REV: (0, 1, 2, 3, 4),
         M_MRTM: (0, 1, 2), M_LPNTPET: (0, 1, 2, 3, 4, 5, 6)}

LAMBDA_F18 = math.log(2.0) / 109.8
LAMBDA_C11 = math.log(2.0) / 20.4

# Feng input parameters (kBq/mL, min): the paper's ranges are in Bq/mL; these
# are the midpoints of those ranges divided by 1000, except kappa_1, whose
# midpoint (500 / min) gives a bolus too short for a 0.2-min grid.
FENG = dict(b1=255.0, b2=105.0, b3=19.0, k1=4.0, k2=1.815, k3=0.0225)

# Prior boxes (lo, hi) per canonical slot K1, k2, k3, k4, vB.
BOX_2TCM_IRR = {0: (0.01, 1.0), 1: (0.01, 1.0), 2: (0.001, 0.3), 3: (0.0, 0.0), 4: (0.0, 0.1)}
BOX_2TCM_REV = {0: (0.01, 1.0), 1: (0.01, 1.0), 2: (0.001, 0.3), 3: (0.0, 0.1), 4: (0.0, 0.1)}
BOX_1TCM = {0: (0.01, 1.0), 1: (0.01, 1.0), 4: (0.0, 0.1)}
# Reference-tissue models, slots R1, k2, k2a, gamma, tD, tP, alpha.  R1/k2/k2a
# ranges are not in the paper (chosen); the activation ranges are the paper's
# simulation ranges.  The tP entry is relative: tP in [tD + 1, 70].
BOX_MRTM = {0: (0.5, 2.0), 1: (0.1, 0.8), 2: (0.01, 0.2)}
BOX_LPNTPET = {0: (0.5, 2.0), 1: (0.1, 0.8), 2: (0.01, 0.2), 3: (0.0, 0.5), 4: (20.0, 50.0), 5: (1.0, 70.0),
               6: (0.25, 4.0)}
REFERENCE = dict(K1=0.1, k2=0.2)

# Frame schedules (durations in minutes).  The paper does not list them for
# these frame counts; all bounds fall on the 0.2-min grid.
SCHED_22x60 = [0.2] * 4 + [0.6] * 4 + [1.2] * 4 + [4.0] * 4 + [6.0] * 6
SCHED_30x50 = [0.2] * 8 + [0.4] * 6 + [1.0] * 6 + [2.0] * 5 + [6.0] * 5
SCHED_40x90 = [0.6] * 10 + [1.2] * 10 + [3.6] * 20


def feng_input(t: np.ndarray, p: dict = FENG) -> np.ndarray:
    """Feng's plasma input C_a(t) (Sec. III-A1), FP64."""
    t = np.asarray(t, dtype=np.float64)
    return ((p["b1"] * t - p["b2"] - p["b3"]) * np.exp(-p["k1"] * t) + p["b2"] * np.exp(-p["k2"] * t)
            + p["b3"] * np.exp(-p["k3"] * t))


def _conv_e0(t, beta, kappa):
    if abs(beta - kappa) < 1e-12:
        return t * np.exp(-beta * t)
    return (np.exp(-kappa * t) - np.exp(-beta * t)) / (beta - kappa)


def _conv_e1(t, beta, kappa):
    if abs(beta - kappa) < 1e-12:
        return 0.5 * t * t * np.exp(-beta * t)
    d = beta - kappa
    return t * np.exp(-kappa * t) / d - (np.exp(-kappa * t) - np.exp(-beta * t)) / d ** 2


def reference_input(t: np.ndarray, p: dict = FENG, r: dict = REFERENCE) -> np.ndarray:
    """Reference-region TAC K1' int_0^t exp(-k2' (t - s)) C_a(s) ds in closed
    form (each term of Feng's input convolved analytically), FP64."""
    t = np.asarray(t, dtype=np.float64)
    b = r["k2"]
    return r["K1"] * (p["b1"] * _conv_e1(t, b, p["k1"]) - (p["b2"] + p["b3"]) * _conv_e0(t, b, p["k1"])
                      + p["b2"] * _conv_e0(t, b, p["k2"]) + p["b3"] * _conv_e0(t, b, p["k3"]))


def frame_times(durations) -> np.ndarray:
    """Contiguous frame bounds [F+1] starting at 0 (fp32)."""
    return np.concatenate([[0.0], np.cumsum(np.asarray(durations, dtype=np.float64))]).astype(np.float32)


def grid(dt: float, t_end: float, reference: bool = False):
    """Node count and the fp32 input function at t_k = k * dt, k = 0..K
    (the plasma input, or the reference-region TAC)."""
    h = float(np.float32(dt))
    K = int(round(t_end / h))
    t = np.arange(K + 1, dtype=np.float64) * h
    return K + 1, (reference_input(t) if reference else feng_input(t)).astype(np.float32)


def box_array(models, boxes=None) -> np.ndarray:
    """[M][8][2] prior box array (unused slots 0)."""
    out = np.zeros((len(models), NSLOT, 2), dtype=np.float64)
    defaults = {M_1TCM: BOX_1TCM, M_2TCM_IRR: BOX_2TCM_IRR, M_2TCM_REV: BOX_2TCM_REV, M_MRTM: BOX_MRTM,
                M_LPNTPET: BOX_LPNTPET}
    for j, m in enumerate(models):
        b = (boxes[j] if boxes is not None else None) or defaults[m]
        for s, (lo, hi) in b.items():
            out[j, s] = (lo, hi)
    return out


def true_params(rng: np.random.Generator, n: int, model: int, box: np.ndarray) -> np.ndarray:
    """fp32 parameter rows [n][8] drawn uniformly from the box; unused slots NaN."""
    th = np.full((n, NSLOT), np.nan, dtype=np.float32)
    for s in SLOTS[model]:
        lo, hi = box[s]
        if model == M_LPNTPET and s == 5:  # tP in [tD + lo, hi]
            th[:, s] = (th[:, 4] + lo + rng.uniform(0.0, 1.0, size=n) * (hi - th[:, 4] - lo)).astype(np.float32)
        else:
            th[:, s] = rng.uniform(lo, hi, size=n).astype(np.float32)
    return th


def frame_mid_and_len(ft: np.ndarray):
    ft = np.asarray(ft, dtype=np.float64)
    return 0.5 * (ft[1:] + ft[:-1]), np.diff(ft)


def add_noise(clean: np.ndarray, ft, eps: np.ndarray, level: float = 0.05,
              lam: float = LAMBDA_F18) -> np.ndarray:
    """Observed TACs: y = C + sqrt(level * C * exp(lam tmid) / dt) * eps (fp32)."""
    tm, dt = frame_mid_and_len(ft)
    c = np.asarray(clean, dtype=np.float64)
    sd = np.sqrt(level * np.clip(c, 0.0, None) * np.exp(lam * tm) / dt)
    return (c + sd * eps).astype(np.float32)


@dataclass
class Workload:
    """One synthetic configuration: grid, frames, models, prior and ABC budget."""
    name: str
    n_voxels: int
    durations: list
    dt: float = 0.2
    models: tuple = (M_2TCM_IRR,)
    n_draws: int = 2000
    accept_frac: float = 0.01
    data_seed: int = 2603014859
    infer_seed: int = 14859
    boxes: list = field(default=None)
    decay_lambda: float = LAMBDA_F18
    reference: bool = False  # the input is a reference-region TAC

    @property
    def frame_times(self) -> np.ndarray:
        return frame_times(self.durations)

    @property
    def t_end(self) -> float:
        return float(np.sum(np.asarray(self.durations, dtype=np.float64)))

    def input_fn(self) -> np.ndarray:
        return grid(self.dt, self.t_end, self.reference)[1]

    def box_array(self) -> np.ndarray:
        return box_array(self.models, self.boxes)

    def truth(self, n: int | None = None, model: int | None = None):
        """True parameters [V][8] and noise draws [V][F], seeded by data_seed."""
        n = self.n_voxels if n is None else n
        rng = np.random.default_rng(self.data_seed)
        model = self.models[0] if model is None else model
        box = box_array([model], None if self.boxes is None else [self.boxes[self.models.index(model)]])[0]
        th = true_params(rng, n, model, box)
        eps = rng.standard_normal((n, len(self.durations)))
        return th, eps

    def truth_mixture(self, n: int | None = None):
        """Irreversible / reversible mixture (total-body configuration): 2TCM
        parameters [V][8] from the reversible box, with k4 = 0 for the
        irreversible half; the reversible mask and noise draws [V][F]."""
        n = self.n_voxels if n is None else n
        rng = np.random.default_rng(self.data_seed)
        th = true_params(rng, n, M_2TCM_REV, box_array([M_2TCM_REV])[0])
        rev = rng.uniform(size=n) < 0.5
        th[~rev, 3] = 0.0
        eps = rng.standard_normal((n, len(self.durations)))
        return th, rev, eps

    def truth_reference(self, n: int | None = None):
        """Reference-tissue configurations: lp-ntPET parameters [V][8] (gamma = 0
        and no activation timing for the null half), the activated mask and
        noise draws [V][F]."""
        n = self.n_voxels if n is None else n
        rng = np.random.default_rng(self.data_seed)
        box = box_array([M_LPNTPET])[0]
        th = true_params(rng, n, M_LPNTPET, box)
        active = rng.uniform(size=n) < 0.5
        th[~active, 3:7] = np.nan
        eps = rng.standard_normal((n, len(self.durations)))
        return th, active, eps


# 1024 voxels (32 x 32), 22 frames over 60 min on a 0.2-min grid, irreversible
# 2TCM prior box, 2000 draws per voxel, 1 % accepted.
CFG_SMALL = Workload("irr2tcm_1024vox_22fr_2000draws", 1024, SCHED_22x60, n_draws=2000,
                     accept_frac=0.01)
# 1,048,576 voxels (128 x 128 x 64), 30 frames over 50 min, 100k per-voxel
# prior draws, 0.1 % accepted.
CFG_LARGE = Workload("irr2tcm_1Mvox_30fr_100kdraws", 1 << 20, SCHED_30x50, n_draws=100_000,
                     accept_frac=0.001)
# Model selection MRTM vs lp-ntPET on a reference-region input: 128 x 128 x 95
# voxels, 40 frames over 90 min, 200k draws per model in one shared bank, 0.1 %
# accepted (n = 400), half of the voxels activated.
CFG_LPNT = Workload("mrtm_lpnt_1.56Mvox_40fr_200kdraws", 128 * 128 * 95, SCHED_40x90,
                    models=(M_MRTM, M_LPNTPET), n_draws=200_000, accept_frac=0.001,
                    decay_lambda=LAMBDA_C11, reference=True)
# Total-body scale: 150 x 150 x 486 voxels, 30 frames over 50 min, half
# irreversible and half reversible 2TCM voxels, one shared bank of 1M draws
# (500k per model), n = 100 accepted, streamed through the GPU in 1M-voxel chunks.
CFG_TBPET = Workload("irrrev_tbpet_10.9Mvox_30fr_1Mbank", 150 * 150 * 486, SCHED_30x50,
                     models=(M_2TCM_IRR, M_2TCM_REV), n_draws=500_000, accept_frac=1e-4)
# Its small streaming case: 3000 voxels, 5000 draws per model, 1 % accepted.
CFG_TBPET_SMALL = Workload("irrrev_3000vox_30fr_10kbank", 3000, SCHED_30x50, models=(M_2TCM_IRR, M_2TCM_REV),
                           n_draws=5000, accept_frac=0.01)
# Its small parity case: 256 voxels, 5000 draws per model, 0.4 % accepted.
CFG_LPNT_SMALL = Workload("mrtm_lpnt_256vox_40fr_5kdraws", 256, SCHED_40x90, models=(M_MRTM, M_LPNTPET),
                          n_draws=5000, accept_frac=0.004, decay_lambda=LAMBDA_C11, reference=True)
