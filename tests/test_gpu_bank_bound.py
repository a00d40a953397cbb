"""The error bound behind the BF16 contraction scan, measured on the matrix cores.

The shared-bank form screens every (voxel, bank row) pair with the weighted L2
distance written as a contraction, d_vg = a_v + sum_k A_vk B_gk with
A_v = [-2 w y, w] and B_g = [x_g, x_g^2] (Alg. 1 line 4 over a shared bank).
The scan computes S ~ sum_k A B from bf16 hi/lo splits with FP32 accumulation,
and its candidate test is exact only if |S - sum_k A B| <= m E for every pair,
E = sum_k |A||B|, m = 2 (3 2^-16 + 3 K 2^-24).  These tests read back the S
that the scan kernel itself computes for every pair (vpet_abc_bank_screen) and
check that inequality against FP64 sums formed here from the same fp32 curves,
fp32 weights and FP64 bank rows, for K = 64, 80 and 96 and for adversarial
voxels: observed curves equal to a bank row (the distance cancels to zero, so
a_v is the whole of |S|), curves a hair away from a bank row, weights spread
over six decades, negative observations, and a large activity scale.
Bank rows come from the oracle's forward model; nothing compared here comes
from the GPU's own arithmetic except S and a_v.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2603_14859_amd as V  # noqa: E402

DEV = torch.device("cuda:0")
H = 0.2
SCHED_48 = [0.2] * 8 + [0.4] * 8 + [1.0] * 12 + [2.0] * 10 + [4.0] * 10


def _m(K):
    return 2.0 * (3.0 * 2.0 ** -16 + 3.0 * K * 2.0 ** -24)


def _case(sched, seed):
    import oracle as ora
    ft = W.frame_times(sched)
    n_nodes, cp = W.grid(H, float(np.sum(sched)))
    F = len(sched)
    models = [W.M_2TCM_IRR, W.M_2TCM_REV]
    _, x = ora.bank(models, W.box_array(models), 1024, seed, cp, H, ft)  # [2048][F] FP64
    N = x.shape[0]
    rng = np.random.default_rng(seed)
    mid, dur = W.frame_mid_and_len(ft)
    # voxels: noisy curves of random truths, exact bank rows, near bank rows,
    # curves with negative frames, and a 1e3 activity scale
    th = W.true_params(rng, 192, W.M_2TCM_IRR, W.box_array([W.M_2TCM_IRR])[0])
    clean = ora.simulate(W.M_2TCM_IRR, th, cp, H, ft)
    noisy = W.add_noise(clean, ft, rng.standard_normal(clean.shape))
    rows = rng.choice(N, size=160, replace=False)
    exact = x[rows[:96]].astype(np.float32)
    near = (x[rows[96:]] * (1.0 + 1e-4 * rng.standard_normal((64, F)))).astype(np.float32)
    neg = noisy[:32] - np.float32(0.5) * noisy[:32].max(axis=1, keepdims=True)
    big = noisy[32:64] * np.float32(1e3)
    y = np.concatenate([noisy, exact, near, neg.astype(np.float32), big.astype(np.float32)]).astype(np.float32)
    Vn = y.shape[0]
    # caller weights (fp32, known exactly here): the Sec. III-A1 inverse
    # variance of the observation, and for a third of the voxels every frame
    # scaled by a factor spread over six decades
    floor = 0.01 * np.maximum(y.max(axis=1, keepdims=True), 1e-3)
    w = dur * np.exp(-np.log(2.0) / 109.8 * mid) / np.maximum(y, floor)
    spread = 10.0 ** rng.uniform(-3.0, 3.0, size=(Vn, F))
    w = np.where((np.arange(Vn) % 3 == 0)[:, None], w * spread, w).astype(np.float32)
    return ft, n_nodes, x, y, w


def _measure(ft, n_nodes, x, y, w):
    F = y.shape[1]
    ld = V.lib.vpet_abc_bank_ld(F)
    xp = np.zeros((x.shape[0], ld))
    xp[:, :F] = x
    s, a = V.bank_screen(torch.from_numpy(y).to(DEV), ft, H, n_nodes, torch.from_numpy(xp).to(DEV),
                         weights=torch.from_numpy(w).to(DEV))
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.float64), a.cpu().numpy(), 2 * ld


@pytest.mark.parametrize("sched", [W.SCHED_30x50, W.SCHED_40x90, SCHED_48], ids=["K64", "K80", "K96"])
def test_contraction_error_within_certified_bound(sched):
    ft, n_nodes, x, y, w = _case(sched, 7 + len(sched))
    s, a, K = _measure(ft, n_nodes, x, y, w)
    yd, wd = y.astype(np.float64), w.astype(np.float64)
    A = np.concatenate([-2.0 * wd * yd, wd], axis=1)           # [V][2F]
    B = np.concatenate([x, x * x], axis=1)                       # [N][2F]
    exact = A @ B.T
    E = np.abs(A) @ np.abs(B).T
    err = np.abs(s - exact)
    m = _m(K)
    ratio = err / (m * E)
    print(f"[bound] K={K} pairs={err.size} max |S - sum AB| / E = {np.max(err / E):.3e} "
          f"(bound m = {m:.3e}; largest share of the bound used {ratio.max():.3f}; "
          f"median {np.median(err / E):.2e})")
    assert np.isfinite(s).all()
    assert np.all(err <= m * E), f"bound exceeded at {np.unravel_index(np.argmax(ratio), ratio.shape)}"
    # a_v = sum w y^2 in FP64 on both sides
    assert np.allclose(a, np.sum(wd * yd * yd, axis=1), rtol=1e-12, atol=0.0)
    # where the distance cancels (observation = bank row) the scan still ranks
    # that row: S + a_v is within the bound of the exact d = 0
    exact_rows = np.arange(192, 192 + 96)
    d_pair = a[exact_rows, None] + s[exact_rows]
    assert np.min(np.abs(d_pair), axis=1).max() <= (m * E[exact_rows]).max()


def test_screen_invalid_voxel_and_limits():
    ft, n_nodes, x, y, w = _case(W.SCHED_30x50, 3)
    y = y[:8].copy()
    y[2, 5] = np.nan
    s, a, _ = _measure(ft, n_nodes, x[:300], y, w[:8])
    assert np.isnan(s[2]).all() and np.isnan(a[2])
    assert np.isfinite(s[[0, 1, 3]]).all()
    big = torch.zeros((4097, V.lib.vpet_abc_bank_ld(30)), dtype=torch.float64, device=DEV)
    with pytest.raises(V.VpetError) as e:
        V.bank_screen(torch.from_numpy(y).to(DEV), ft, H, n_nodes, big)
    assert e.value.status == V.E_LIMIT
