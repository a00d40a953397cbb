"""Pins for the oracle's forward model (Eq. (1)-(2) with the linear-input,
exact-exponential discretisation) and its frame averaging.

Each check is against something the mathematics fixes, not against the
oracle's own formulas:
  * the step is exact for piecewise-linear input (constant and ramp closed forms);
  * it converges at order 2 to the analytic convolution with Feng's input;
  * the model TACs agree with a fine RK4 integration of the ODE of Eq. (1);
  * the irreversible rate-0 amplitude is Ki (Patlak slope for a constant input);
  * the trapezoid frame average is exact for linear and has the known error for
    quadratic node data.
"""
import math

import numpy as np
import pytest

import workloads as W
from closed_forms import feng_conv_exp, feng_integral, rk4_2tcm_nodes


def test_step_coefficients_series_and_limits(ora):
    h = 0.2
    for beta in [1e-14, 1e-6, 4.99e-3, 5.01e-3, 0.011, 0.3, 0.499, 0.501, 1.3, 7.0]:
        e, a, b = ora.step_coeffs(beta, h)
        x = beta * h
        assert e == pytest.approx(np.exp(-x), rel=1e-15)
        # a + b integrates exp(-beta s) over one step.
        assert a + b == pytest.approx(-np.expm1(-x) / beta if beta > 0 else h, rel=1e-12)
    # beta -> 0 is the trapezoid rule.
    e, a, b = ora.step_coeffs(0.0, h)
    assert (e, a, b) == (1.0, h / 2, h / 2)
    # the series branch (x < 0.1) and the closed-form branch agree across the switch
    _, a1, b1 = ora.step_coeffs(0.1 * (1 - 1e-12) / h, h)
    _, a2, b2 = ora.step_coeffs(0.1 / h, h)
    assert a1 == pytest.approx(a2, rel=1e-13) and b1 == pytest.approx(b2, rel=1e-13)
    # and both match high-precision values (mpmath-free: a rational Taylor sum
    # in Python floats of 40 terms at x = 0.05 and x = 0.2)
    for x in (0.05, 0.2):
        beta = x / h
        _, a, b = ora.step_coeffs(beta, h)
        ta = sum((-1) ** m * (m - 1) / math.factorial(m) * x ** (m - 2) for m in range(2, 42))
        tb = sum((-1) ** m / math.factorial(m) * x ** (m - 2) for m in range(2, 42))
        assert a == pytest.approx(h * ta, rel=1e-14) and b == pytest.approx(h * tb, rel=1e-14)


@pytest.mark.parametrize("beta", [0.0, 1e-5, 0.011, 0.3, 1.3])
def test_exact_for_constant_and_ramp_input(ora, beta):
    h, K = 0.2, 300
    t = np.arange(K + 1) * h
    const = ora.convolve_exp(beta, np.full(K + 1, 2.5), h)
    ramp = ora.convolve_exp(beta, 0.7 * t, h)
    if beta == 0.0:
        want_c, want_r = 2.5 * t, 0.7 * t * t / 2
    else:
        want_c = 2.5 * (-np.expm1(-beta * t)) / beta
        want_r = 0.7 * (t / beta + np.expm1(-beta * t) / beta ** 2)
    assert np.allclose(const, want_c, rtol=1e-12, atol=1e-12 * np.abs(want_c).max())
    assert np.allclose(ramp, want_r, rtol=1e-10, atol=1e-11 * np.abs(want_r).max())


@pytest.mark.parametrize("beta", [0.011, 0.3, 1.3])
def test_second_order_convergence_to_feng_closed_form(ora, beta):
    errs = []
    T = 60.0
    for h in [0.2, 0.1, 0.05, 0.025]:
        K = int(round(T / h))
        t = np.arange(K + 1) * h
        num = ora.convolve_exp(beta, W.feng_input(t), h)
        ex = feng_conv_exp(t, beta, W.FENG)
        errs.append(np.abs(num - ex).max() / np.abs(ex).max())
    ratios = [errs[j] / errs[j + 1] for j in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)
    # beta = 0 is the cumulative trapezoid integral of the input
    h = 0.05
    t = np.arange(int(T / h) + 1) * h
    q = ora.convolve_exp(0.0, W.feng_input(t), h)
    assert np.abs(q - feng_integral(t, W.FENG)).max() < 1e-3 * np.abs(q).max()


@pytest.mark.parametrize("theta", [
    (0.5, 0.3, 0.05, 0.0, 0.05),      # irreversible
    (0.9, 0.011, 0.001, 0.0, 0.0),    # slowest irreversible corner of the box
    (0.2, 1.0, 0.3, 0.0, 0.1),        # fastest corner
    (0.5, 0.3, 0.05, 0.02, 0.05),     # reversible
    (0.7, 0.05, 0.25, 0.1, 0.03),     # reversible, strong exchange
    (0.4, 0.6, 0.001, 0.09, 0.0),     # reversible, weak trapping
])
def test_2tcm_matches_rk4(ora, theta):
    h, K = 0.2, 300
    cp = W.feng_input(np.arange(K + 1) * h)
    th = np.full(8, np.nan)
    th[[0, 1, 2, 3, 4]] = theta
    model = W.M_2TCM_IRR if theta[3] == 0.0 else W.M_2TCM_REV
    got = ora.simulate_nodes(model, th, cp, h)
    want = rk4_2tcm_nodes(theta, cp, h)
    assert np.abs(got - want).max() < 1e-9 * np.abs(want).max()
    if model == W.M_2TCM_IRR:
        # the reversible form with k4 -> 0 reduces to the irreversible one
        th2 = th.copy()
        th2[3] = 1e-13
        rev = ora.simulate_nodes(W.M_2TCM_REV, th2, cp, h)
        assert np.abs(rev - got).max() < 1e-9 * np.abs(got).max()


def test_1tcm_matches_rk4(ora):
    h, K = 0.2, 300
    cp = W.feng_input(np.arange(K + 1) * h)
    th = np.full(8, np.nan)
    th[[0, 1, 4]] = (0.6, 0.15, 0.04)
    got = ora.simulate_nodes(W.M_1TCM, th, cp, h)
    # 1TCM is the 2TCM with k3 = k4 = 0
    want = rk4_2tcm_nodes((0.6, 0.15, 0.0, 0.0, 0.04), cp, h)
    assert np.abs(got - want).max() < 1e-9 * np.abs(want).max()


def test_irreversible_rate0_amplitude_is_ki(ora):
    # Constant input c: C_T(t) - (1 - vB) Ki c t tends to a constant (Patlak).
    h, K = 0.2, 3000
    c = 3.0
    K1, k2, k3, vB = 0.4, 0.2, 0.07, 0.05
    th = np.full(8, np.nan)
    th[[0, 1, 2, 4]] = (K1, k2, k3, vB)
    nodes = ora.simulate_nodes(W.M_2TCM_IRR, th, np.full(K + 1, c), h)
    slope = (nodes[-1] - nodes[-501]) / (500 * h)
    ki = K1 * k3 / (k2 + k3)
    assert slope == pytest.approx((1 - vB) * ki * c, rel=1e-10)


def test_frame_average_linear_and_quadratic(ora):
    h = 0.2
    t = np.arange(301) * h
    kf = ora.frame_nodes(W.frame_times(W.SCHED_22x60), h, 301)
    a, b = t[kf[:-1]], t[kf[1:]]
    lin = ora.frame_average(2.0 + 3.0 * t, kf)
    assert np.allclose(lin, 2.0 + 3.0 * 0.5 * (a + b), rtol=1e-13)
    quad = ora.frame_average(t * t, kf)
    # composite trapezoid error for t^2 over [a, b]: (h^2/12) (f'(b) - f'(a)) = h^2 (b - a)/6
    exact = (b ** 3 - a ** 3) / (3 * (b - a)) + h * h / 6
    assert np.allclose(quad, exact, rtol=1e-12)


def test_frame_nodes_validation(ora):
    with pytest.raises(ValueError):
        ora.frame_nodes(np.array([0.0, 0.3, 1.0], dtype=np.float32), 0.2, 301)
    with pytest.raises(ValueError):
        ora.frame_nodes(np.array([0.0, 1.0, 1.0], dtype=np.float32), 0.2, 301)
    with pytest.raises(ValueError):
        ora.frame_nodes(np.array([0.0, 61.0], dtype=np.float32), 0.2, 301)
