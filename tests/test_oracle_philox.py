"""Pins for the oracle's draws (Alg. 1, lines 1-2): Philox4x32-10 and u -> theta.

* Philox is checked word for word against rocRAND's Philox4x32-10 engine, a
  library routine compiled here from the installed headers and run on the CPU.
* The unit map and the fp32 theta map are checked against exact rational
  arithmetic.
* Uniformity: chi-square over 256 bins and the first two moments.
"""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("rr") / "philox_ref")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "helpers", "rocrand_philox_ref.cpp"), "-o", exe],
                   check=True, capture_output=True)

    def run(seeds, ctrs):
        lines = "".join(f"{int(s)} {c[0]} {c[1]} {c[2]} {c[3]}\n" for s, c in zip(seeds, ctrs))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w, 16) for w in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint32)

    return run


def test_philox_matches_rocrand(ora, rocrand_ref):
    rng = np.random.default_rng(1)
    n = 3000
    # rocRAND positions its engine by a 64-bit "offset" of 4 * (c0 + 2^32 c1),
    # so c1 stays below 2^30 here; c2 and c3 range freely.
    ctr = np.stack([rng.integers(0, 2**32, n), rng.integers(0, 2**30, n),
                    rng.integers(0, 2**32, n), rng.integers(0, 2**32, n)], axis=1).astype(np.uint32)
    ctr[:8] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1],
               [2**32 - 1, 0, 0, 0], [7, 3, 0, (2 << 16) | 1], [123, 456, 0, 0]]
    seeds = rng.integers(0, 2**63, n, dtype=np.uint64)
    seeds[:4] = [0, 1, 14859, 2**63 + 5]
    want = rocrand_ref(seeds, ctr)
    got = np.stack([ora.philox(ctr[j:j + 1], int(seeds[j]))[0] for j in range(n)])
    assert np.array_equal(got, want)


def test_philox_uniformity(ora):
    n = 1 << 18
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n)
    ctr[:, 1] = 17
    w = ora.philox(ctr, 14859)
    u = (w >> 8).astype(np.float64) / 2**24
    for j in range(4):
        uj = u[:, j]
        assert abs(uj.mean() - 0.5) < 5 * np.sqrt(1 / 12 / n)
        assert abs(uj.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / n)
        counts = np.bincount((uj * 256).astype(int), minlength=256)
        chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
        assert chi2 < 255 + 6 * np.sqrt(2 * 255)  # far tail of chi2(255)
    c = np.corrcoef(u.T)
    assert np.all(np.abs(c - np.eye(4)) < 5 / np.sqrt(n))


def _round_f32(x: Fraction) -> np.float32:
    """Round an exact rational to the nearest fp32 (ties to even)."""
    f = np.float32(float(x))
    best, berr = None, None
    for cand in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        err = abs(Fraction(float(cand)) - x)
        if berr is None or err < berr or (err == berr and (cand.view(np.uint32) & 1) == 0):
            best, berr = cand, err
    return best


def test_theta_map_exact(ora):
    models = np.array([2, 4, 1], dtype=np.uint32)
    boxes = np.zeros((3, 8, 2))
    boxes[0, [0, 1, 2, 4]] = [(0.01, 1.0), (0.01, 1.0), (0.001, 0.3), (0.0, 0.1)]
    boxes[1, [0, 1, 2, 3, 4]] = [(0.01, 1.0), (0.013, 0.9), (0.001, 0.3), (0.0, 0.1), (0.03, 0.2)]
    boxes[2, [0, 1, 4]] = [(0.5, 0.5), (1e-3, 2.0), (0.0, 0.1)]
    slots = {0: [0, 1, 2, 4], 1: [0, 1, 2, 3, 4], 2: [0, 1, 4]}
    rng = np.random.default_rng(2)
    n = 600
    v = rng.integers(0, 2**32, n)
    i = rng.integers(0, 2**32, n)
    m = rng.integers(0, 3, n).astype(np.int32)
    words, u, theta = ora.draws(models, boxes, 99, v, i, m)
    for j in range(n):
        mj = int(m[j])
        nb = (len(slots[mj]) + 3) // 4
        ref_words = np.concatenate([ora.philox(np.array([[i[j], v[j], 0, (mj << 16) | b]], dtype=np.uint32), 99)[0]
                                    for b in range(nb)])
        assert np.array_equal(words[j, :4 * nb], ref_words)
        for p, s in enumerate(slots[mj]):
            uu = Fraction(int(ref_words[p]) >> 8, 2**24)
            assert Fraction(float(u[j, p])) == uu
            lo, hi = boxes[mj, s]
            exact = Fraction(float(np.float32(hi - lo))) * uu + Fraction(float(np.float32(lo)))
            assert theta[j, s] == _round_f32(exact)
        unused = [s for s in range(8) if s not in slots[mj]]
        assert np.all(np.isnan(theta[j, unused]))
    # a fixed parameter (lo == hi) is drawn exactly
    assert np.all(theta[m == 2, 0] == np.float32(0.5))
