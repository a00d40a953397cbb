"""Pins for the oracle's reference-tissue models: MRTM and lp-ntPET
(Sec. II-A2, Eq. (3)-(4)), whose input is the reference-region TAC C_r.

Each check is against something the mathematics or the paper fixes:
  * the activation g is 0 up to t_D and peaks at 1 at t_P;
  * MRTM is exact for piecewise-linear C_r (constant and ramp closed forms);
  * lp-ntPET with gamma = 0 is MRTM;
  * lp-ntPET agrees with a fine RK4 integration of the ODE, at order 2;
  * both satisfy the integral form of Eq. (3)-(4) to second order (this pins
    the signs and factors of every term against the paper's equation);
  * the relative t_P box of the draws is exact in fp32 and inside [tD + lo, hi];
  * BP_ND = k2 / k2a - 1 per accepted sample; model selection prefers
    lp-ntPET for an activated curve and not for a flat one.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from closed_forms import rk4_reference_nodes
from test_oracle_philox import _round_f32

THETA_ACT = (1.2, 0.35, 0.08, 0.3, 20.0, 32.0, 2.0)   # R1, k2, k2a, gamma, tD, tP, alpha


def _theta8(t7):
    th = np.full(8, np.nan)
    th[:len(t7)] = t7
    return th


def _cr_analytic(t):
    """A smooth reference-like curve (rise and slow washout), kBq/mL."""
    t = np.asarray(t, dtype=np.float64)
    return 8.0 * (1.0 - np.exp(-0.9 * t)) * np.exp(-0.02 * t) + 0.3 * t * np.exp(-0.1 * t)


def test_gamma_variate_shape(ora):
    tD, tP = 20.0, 31.0
    for alpha in (0.25, 1.0, 4.0):
        assert ora.gamma_variate(tD - 1.0, tD, tP, alpha) == 0.0
        assert ora.gamma_variate(tD, tD, tP, alpha) == 0.0
        assert ora.gamma_variate(tP, tD, tP, alpha) == pytest.approx(1.0, abs=1e-15)
        ts = np.linspace(tD + 0.01, 90.0, 4001)
        g = np.array([ora.gamma_variate(t, tD, tP, alpha) for t in ts])
        assert g.max() <= 1.0 + 1e-15
        assert abs(ts[np.argmax(g)] - tP) < 0.05
        assert np.all(g > 0.0)


@pytest.mark.parametrize("k2a", [1e-4, 0.03, 0.4])
def test_mrtm_exact_for_constant_and_ramp_reference(ora, k2a):
    h, K = 0.2, 300
    t = np.arange(K + 1) * h
    R1, k2 = 1.3, 0.25
    th = _theta8((R1, k2, k2a))
    c = 3.5
    got = ora.simulate_nodes(ora.M_MRTM, th, np.full(K + 1, c), h)
    ref = R1 * c + (k2 - R1 * k2a) * c * (-np.expm1(-k2a * t)) / k2a
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
    got = ora.simulate_nodes(ora.M_MRTM, th, t, h)
    ref = R1 * t + (k2 - R1 * k2a) * (t / k2a + np.expm1(-k2a * t) / k2a ** 2)
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_lpntpet_with_zero_gamma_is_mrtm(ora):
    h = 0.2
    cr = _cr_analytic(np.arange(451) * h)
    th = _theta8(THETA_ACT)
    th[3] = 0.0
    a = ora.simulate_nodes(ora.M_LPNTPET, th, cr, h)
    b = ora.simulate_nodes(ora.M_MRTM, _theta8(THETA_ACT[:3]), cr, h)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    # activation only after tD: identical curves up to the first step past tD
    th[3] = 0.3
    c = ora.simulate_nodes(ora.M_LPNTPET, th, cr, h)
    kD = int(round(THETA_ACT[4] / h))
    assert np.allclose(c[:kD + 1], b[:kD + 1], rtol=1e-12, atol=1e-12)
    assert np.all(c[kD + 5:] < b[kD + 5:])  # displacement lowers the target TAC


def test_lpntpet_converges_to_rk4_at_second_order(ora):
    T = 60.0
    errs = []
    for h in (0.4, 0.2, 0.1):
        K = int(round(T / h))
        t = np.arange(K + 1) * h
        cr = _cr_analytic(t)
        got = ora.simulate_nodes(ora.M_LPNTPET, _theta8(THETA_ACT), cr, h)
        ref = rk4_reference_nodes(THETA_ACT, cr, h, sub=16)
        errs.append(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    assert errs[1] < 1e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.4 < a / b < 4.6, errs


@pytest.mark.parametrize("model", ["mrtm", "lpnt"])
def test_integral_form_of_eq3_holds_to_second_order(ora, model):
    """C_t = R1 C_r + k2 int C_r - k2a int C_t - gamma int C_t g  (Eq. (3)-(4)),
    integrals by the trapezoid rule on the grid: the residual shrinks as h^2."""
    T = 60.0
    res = []
    for h in (0.4, 0.2, 0.1):
        K = int(round(T / h))
        t = np.arange(K + 1) * h
        cr = _cr_analytic(t)
        if model == "mrtm":
            th, gam = _theta8(THETA_ACT[:3]), 0.0
            ct = ora.simulate_nodes(ora.M_MRTM, th, cr, h)
        else:
            th, gam = _theta8(THETA_ACT), THETA_ACT[3]
            ct = ora.simulate_nodes(ora.M_LPNTPET, th, cr, h)
        R1, k2, k2a = THETA_ACT[:3]
        g = np.array([ora.gamma_variate(tt, *THETA_ACT[4:6], THETA_ACT[6]) for tt in t])

        def cumtrap(v):
            return np.concatenate([[0.0], np.cumsum(0.5 * h * (v[1:] + v[:-1]))])

        rhs = R1 * cr + k2 * cumtrap(cr) - k2a * cumtrap(ct) - gam * cumtrap(ct * g)
        res.append(np.max(np.abs(ct - rhs)) / np.max(np.abs(ct)))
    assert res[1] < 1e-3
    for a, b in zip(res, res[1:]):
        assert 3.0 < a / b < 5.0, res


def test_lpntpet_relative_tp_box_is_exact(ora):
    models = np.array([ora.M_MRTM, ora.M_LPNTPET], dtype=np.uint32)
    boxes = np.zeros((2, 8, 2))
    boxes[0, :3] = [(0.5, 2.0), (0.1, 0.8), (0.01, 0.2)]
    boxes[1, :7] = [(0.5, 2.0), (0.1, 0.8), (0.01, 0.2), (0.0, 0.5), (20.0, 50.0), (1.0, 70.0), (0.25, 4.0)]
    rng = np.random.default_rng(5)
    n = 400
    v = rng.integers(0, 2**32, n)
    i = rng.integers(0, 2**32, n)
    m = rng.integers(0, 2, n).astype(np.int32)
    words, u, theta = ora.draws(models, boxes, 7, v, i, m, stream=1)
    for j in range(n):
        mj = int(m[j])
        np_ = 3 if mj == 0 else 7
        assert np.all(np.isnan(theta[j, np_:]))
        for s in range(np_):
            uu = Fraction(int(words[j, s]) >> 8, 2**24)
            lo, hi = boxes[mj, s]
            if mj == 1 and s == 5:
                lo_f = np.float32(theta[j, 4] + np.float32(lo))
                exact = Fraction(float(np.float32(np.float32(hi) - lo_f))) * uu + Fraction(float(lo_f))
            else:
                exact = Fraction(float(np.float32(hi - lo))) * uu + Fraction(float(np.float32(lo)))
            assert theta[j, s] == _round_f32(exact)
        if mj == 1:
            assert theta[j, 4] + 1.0 - 1e-5 <= theta[j, 5] <= 70.0


def test_bp_nd_summary_and_model_selection(ora):
    cfg = W.CFG_LPNT_SMALL
    ft, cr = cfg.frame_times, cfg.input_fn()
    boxes = cfg.box_array()
    models = list(cfg.models)
    # p = 1: the BP_ND mean is the mean of k2/k2a - 1 over every draw of the model
    y0 = ora.simulate(ora.M_MRTM, np.array([[1.0, 0.3, 0.05] + [np.nan] * 5], dtype=np.float32), cr, cfg.dt, ft)
    y0 = y0.astype(np.float32)
    o = ora.infer_bank(y0, ft, cr, cfg.dt, models, boxes, 300, 1.0, 3, lam=cfg.decay_lambda)
    th, _ = ora.bank(models, boxes, 300, 3, cr, cfg.dt, ft)
    bp = th[:300, 1].astype(np.float64) / th[:300, 2].astype(np.float64) - 1.0
    assert o["moments"][0, 0, 7, 0] == pytest.approx(bp.mean(), rel=1e-12)
    assert np.isnan(o["moments"][0, 0, 3:7]).all()
    # noise-free activated vs flat curves against one bank: lp-ntPET is
    # preferred for the activated curve only
    act = np.array([list(THETA_ACT) + [np.nan]], dtype=np.float32)
    act[0, 3] = 0.45
    null = np.array([[1.2, 0.35, 0.08] + [np.nan] * 5], dtype=np.float32)
    y = np.vstack([ora.simulate(ora.M_LPNTPET, act, cr, cfg.dt, ft),
                   ora.simulate(ora.M_MRTM, null, cr, cfg.dt, ft)]).astype(np.float32)
    o = ora.infer_bank(y, ft, cr, cfg.dt, models, boxes, 20000, 0.002, 11, lam=cfg.decay_lambda)
    p_act, p_null = o["model_prob"][0, 1], o["model_prob"][1, 1]
    assert p_act > 0.75 and p_act > p_null + 0.25, (p_act, p_null)
