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
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

M_1TCM = 1
M_2TCM_IRR = 2
M_2TCM_REV = 4
NSLOT = 8
SLOTS = {M_1TCM: (0, 1, 4), M_2TCM_IRR: (0, 1, 2, 4), M_2TCM_REV: (0, 1, 2, 3, 4)}

LAMBDA_F18 = math.log(2.0) / 109.8

# Feng input parameters (kBq/mL, min): the paper's ranges are in Bq/mL; these
# are the midpoints of those ranges divided by 1000, except kappa_1, whose
# midpoint (500 / min) gives a bolus too short for a 0.2-min grid.
FENG = dict(b1=255.0, b2=105.0, b3=19.0, k1=4.0, k2=1.815, k3=0.0225)

# Prior boxes (lo, hi) per canonical slot K1, k2, k3, k4, vB.
BOX_2TCM_IRR = {0: (0.01, 1.0), 1: (0.01, 1.0), 2: (0.001, 0.3), 3: (0.0, 0.0), 4: (0.0, 0.1)}
BOX_2TCM_REV = {0: (0.01, 1.0), 1: (0.01, 1.0), 2: (0.001, 0.3), 3: (0.0, 0.1), 4: (0.0, 0.1)}
BOX_1TCM = {0: (0.01, 1.0), 1: (0.01, 1.0), 4: (0.0, 0.1)}

# Frame schedules (durations in minutes).  The paper does not list them for
# these frame counts; all bounds fall on the 0.2-min grid.
SCHED_22x60 = [0.2] * 4 + [0.6] * 4 + [1.2] * 4 + [4.0] * 4 + [6.0] * 6
SCHED_30x50 = [0.2] * 8 + [0.4] * 6 + [1.0] * 6 + [2.0] * 5 + [6.0] * 5


def feng_input(t: np.ndarray, p: dict = FENG) -> np.ndarray:
    """Feng's plasma input C_a(t) (Sec. III-A1), FP64."""
    t = np.asarray(t, dtype=np.float64)
    return ((p["b1"] * t - p["b2"] - p["b3"]) * np.exp(-p["k1"] * t) + p["b2"] * np.exp(-p["k2"] * t)
            + p["b3"] * np.exp(-p["k3"] * t))


def frame_times(durations) -> np.ndarray:
    """Contiguous frame bounds [F+1] starting at 0 (fp32)."""
    return np.concatenate([[0.0], np.cumsum(np.asarray(durations, dtype=np.float64))]).astype(np.float32)


def grid(dt: float, t_end: float):
    """Node count and the fp32 input function at t_k = k * dt, k = 0..K."""
    h = float(np.float32(dt))
    K = int(round(t_end / h))
    t = np.arange(K + 1, dtype=np.float64) * h
    return K + 1, feng_input(t).astype(np.float32)


def box_array(models, boxes=None) -> np.ndarray:
    """[M][8][2] prior box array (unused slots 0)."""
    out = np.zeros((len(models), NSLOT, 2), dtype=np.float64)
    defaults = {M_1TCM: BOX_1TCM, M_2TCM_IRR: BOX_2TCM_IRR, M_2TCM_REV: BOX_2TCM_REV}
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

    @property
    def frame_times(self) -> np.ndarray:
        return frame_times(self.durations)

    @property
    def t_end(self) -> float:
        return float(np.sum(np.asarray(self.durations, dtype=np.float64)))

    def input_fn(self) -> np.ndarray:
        return grid(self.dt, self.t_end)[1]

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


# 1024 voxels (32 x 32), 22 frames over 60 min on a 0.2-min grid, irreversible
# 2TCM prior box, 2000 draws per voxel, 1 % accepted.
CFG_SMALL = Workload("irr2tcm_1024vox_22fr_2000draws", 1024, SCHED_22x60, n_draws=2000,
                     accept_frac=0.01)
# 1,048,576 voxels (128 x 128 x 64), 30 frames over 50 min, 100k per-voxel
# prior draws, 0.1 % accepted.
CFG_LARGE = Workload("irr2tcm_1Mvox_30fr_100kdraws", 1 << 20, SCHED_30x50, n_draws=100_000,
                     accept_frac=0.001)
